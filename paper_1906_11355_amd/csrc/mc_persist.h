// Ticket protocol of the persistent batched launch: one launch runs every
// work unit of every pass of every volume of a batch.  Plain data and
// functions shared by the device kernel and a host model of the protocol
// (host threads standing in for work-groups), templated on the atomic
// operations, so that both run the very same decisions.
//
// Tickets are handed out in order from one counter.  Their order is phase
// major (all range units of all volumes, then all histogram units, then all
// clip units, then all interpolation units; volumes in batch order inside a
// phase), which is a topological order of the dependencies: a unit of pass p
// of volume v needs every unit of pass p - 1 of v (the histograms need the
// range partials; a kernel's clip needs all histogram partials of its
// column; a cell's interpolation needs the LUTs of its corner kernels; all
// units of the volume's previous pass cover each of these).  A work-group
// finishes its ticket before taking another, so the lowest unfinished
// ticket never waits on anything unfinished: the queue cannot deadlock.
//
// Every wait is bounded anyway.  A wait polls the volume's completion
// counter of the previous pass and one abort word of the whole run; after
// max_spins polls it sets the abort word and gives up.  Only units that ran
// count, so once the word is set a unit whose producers were skipped never
// runs: its wait ends on the word.  A run that cannot complete still drains
// its tickets and the kernel ends normally; the word tells the host which
// ticket gave up.
#pragma once
#include "mc_desc.h"

#define MC_NO_TICKET 0xffffffffu

// Head of a persistent batch table (device memory, uploaded per call); the
// unit prefix sums follow it: pre[MC_PHASES][nvol + 1] (uint32).
struct McPersistHdr {
    uint32_t total;                        // tickets of the whole run
    uint32_t nvol;
    uint32_t max_spins;                    // polls of one wait before the run aborts
    uint32_t abort_at;                     // test hook: this ticket's wait aborts the run
    uint32_t phase_start[MC_PHASES + 1];   // first ticket of each pass; [MC_PHASES] = total
    uint32_t pad_[3];
};

// Words of a run (cleared before each launch): head, abort, then the
// completion counters done[MC_PHASES][nvol].
#define MC_PQ_HEAD 0
#define MC_PQ_ABORT 1
#define MC_PQ_DONE 2

MC_HD uint32_t mc_persist_words(uint32_t nvol) { return MC_PQ_DONE + MC_PHASES * nvol; }

// What the persistent kernel receives (device pointers into the batch table).
struct McPersistSrc {
    const McPersistHdr *hdr;
    const uint32_t *pre;      // [MC_PHASES][nvol + 1] unit prefix sums
    const McVol *vols;        // [nvol]
    uint32_t *q;              // [mc_persist_words(nvol)] run words
};

struct McTicket {
    uint32_t phase, vol, unit;
};

// Pass, volume and unit of ticket t < total.
MC_HD McTicket mc_ticket(const McPersistHdr &h, const uint32_t *pre, uint32_t t)
{
    uint32_t ph = 0;
    while (ph + 1 < MC_PHASES && t >= h.phase_start[ph + 1]) ++ph;
    const uint32_t r = t - h.phase_start[ph];
    const uint32_t *pp = pre + ph * (h.nvol + 1);
    const uint32_t v = mc_batch_volume(pp, h.nvol, r);
    McTicket k;
    k.phase = ph;
    k.vol = v;
    k.unit = r - pp[v];
    return k;
}

// Units of pass ph of volume v.
MC_HD uint32_t mc_persist_units(const McPersistHdr &h, const uint32_t *pre, uint32_t ph, uint32_t v)
{
    const uint32_t *pp = pre + ph * (h.nvol + 1);
    return pp[v + 1] - pp[v];
}

// Wait until ticket t may run.  Returns true to run its unit, false to skip
// it (the run was aborted, by this wait or an earlier one).  A: the atomic
// operations -- peek reads a word cheaply but possibly late (an older value:
// counters only grow, so a peeked count at or above the need is final),
// poll reads it coherently (dearer), set_abort stores the first abort only,
// sleep pauses between polls.  Most tickets find their pass done already
// and pass on two peeks; only a real wait polls.
template <class A>
MC_HD bool mc_persist_wait(const McPersistHdr &h, const uint32_t *pre, uint32_t *q, const McTicket &k,
                           uint32_t t)
{
    if (t == h.abort_at) {
        A::set_abort(&q[MC_PQ_ABORT], t + 1);
        return false;
    }
    if (A::peek(&q[MC_PQ_ABORT])) return false;
    if (k.phase == 0) return true;
    const uint32_t need = mc_persist_units(h, pre, k.phase - 1, k.vol);
    uint32_t *cnt = &q[MC_PQ_DONE + (k.phase - 1) * h.nvol + k.vol];
    if (A::peek(cnt) >= need) return true;
    for (uint32_t spins = 0;; ++spins) {
        if (A::poll(cnt) >= need) return true;
        if (A::poll(&q[MC_PQ_ABORT])) return false;
        if (spins >= h.max_spins) {
            A::set_abort(&q[MC_PQ_ABORT], t + 1);
            return false;
        }
        A::sleep();
    }
}

// Counter a ticket whose unit ran increments.
MC_HD uint32_t *mc_persist_done(const McPersistHdr &h, uint32_t *q, const McTicket &k)
{
    return &q[MC_PQ_DONE + k.phase * h.nvol + k.vol];
}
