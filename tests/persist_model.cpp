// Host model of the persistent batched launch's ticket protocol: host
// threads stand in for work-groups and run the very protocol functions of
// mc_persist.h (ticket decoding, bounded waits, abort word, completion
// counters) on a real batch table image written by the library
// (mclahe_batched_table).  A unit's "work" marks it done after an optional
// random delay; before running, every unit checks that all units of its
// volume's previous pass are marked, which is what the GPU units rely on.
//
//   persist_model <image file> <workers> <max delay us> <max spins>
//                 <abort ticket | -1> <stall ticket | -1> <stall ms> <mutant 0|1>
//
// Prints: aborted-word tickets-taken units-run violations duplicates missing
// elapsed-ms.  mutant 1 makes every counter poll read one more finished
// unit than there is (a planted protocol mistake the checks must catch).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "mc_desc.h"
#include "mc_persist.h"

static uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static bool g_mutant = false;
static uint32_t *g_done_lo = nullptr, *g_done_hi = nullptr;   // the completion counters' words

// peek is a relaxed load that reads as zero half of the time: on the device
// it may be late (an older value), which the protocol must tolerate, and a
// zero is the oldest value any run word had.
static thread_local std::mt19937 t_rng(7);
struct HostAtomics {
    static uint32_t peek(uint32_t *p)
    {
        if (t_rng() & 1u) return 0u;
        const uint32_t v = __atomic_load_n(p, __ATOMIC_RELAXED);
        return (g_mutant && p >= g_done_lo && p < g_done_hi) ? v + 1 : v;
    }
    static uint32_t poll(uint32_t *p)
    {
        const uint32_t v = __atomic_load_n(p, __ATOMIC_ACQUIRE);
        return (g_mutant && p >= g_done_lo && p < g_done_hi) ? v + 1 : v;
    }
    static void set_abort(uint32_t *p, uint32_t v)
    {
        uint32_t z = 0;
        __atomic_compare_exchange_n(p, &z, v, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE);
    }
    static void sleep() { std::this_thread::yield(); }
};

int main(int argc, char **argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: %s image workers delay_us max_spins abort_ticket stall_ticket stall_ms mutant\n",
                argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<char> img;
    {
        char buf[1 << 16];
        size_t r;
        while ((r = fread(buf, 1, sizeof buf, f)) > 0) img.insert(img.end(), buf, buf + r);
        fclose(f);
    }
    const int workers = atoi(argv[2]);
    const int delay_us = atoi(argv[3]);
    const long long spins = atoll(argv[4]);
    const long long abort_ticket = atoll(argv[5]);
    const long long stall_ticket = atoll(argv[6]);
    const int stall_ms = atoi(argv[7]);
    g_mutant = atoi(argv[8]) != 0;

    const McBatchHdr *bh = (const McBatchHdr *)img.data();
    McPersistHdr h;
    memcpy(&h, img.data() + bh->o_persist, sizeof h);
    const uint32_t *pre = (const uint32_t *)(img.data() + a256(bh->o_persist + sizeof(McPersistHdr)));
    if (h.nvol != bh->nvol || h.phase_start[MC_PHASES] != h.total) return 3;
    if (spins >= 0) h.max_spins = (uint32_t)spins;
    h.abort_at = abort_ticket >= 0 ? (uint32_t)abort_ticket : MC_NO_TICKET;

    std::vector<uint32_t> q(mc_persist_words(h.nvol), 0u);
    g_done_lo = &q[MC_PQ_DONE];
    g_done_hi = q.data() + q.size();
    // marks[ph][v][u]: times unit u of pass ph of volume v ran
    std::vector<std::vector<std::vector<std::atomic<uint8_t>>>> marks(MC_PHASES);
    for (int ph = 0; ph < MC_PHASES; ++ph) {
        marks[ph] = std::vector<std::vector<std::atomic<uint8_t>>>(h.nvol);
        for (uint32_t v = 0; v < h.nvol; ++v) {
            marks[ph][v] = std::vector<std::atomic<uint8_t>>(mc_persist_units(h, pre, ph, v));
            for (auto &m : marks[ph][v]) m.store(0);
        }
    }
    std::atomic<uint64_t> ran(0), violations(0);
    const auto t0 = std::chrono::steady_clock::now();
    auto worker = [&](int id) {
        std::mt19937 rng(1234u + (uint32_t)id);
        for (;;) {
            const uint32_t t = __atomic_fetch_add(&q[MC_PQ_HEAD], 1u, __ATOMIC_RELAXED);
            if (t >= h.total) return;
            const McTicket k = mc_ticket(h, pre, t);
            const bool go = mc_persist_wait<HostAtomics>(h, pre, q.data(), k, t);
            // the kernel's acquire after the wait (a peek is a relaxed load)
            std::atomic_thread_fence(std::memory_order_acquire);
            if (go) {
                if (k.phase > 0) {   // every unit of the previous pass must have run
                    for (auto &m : marks[k.phase - 1][k.vol])
                        if (m.load(std::memory_order_relaxed) == 0) {
                            violations++;
                            break;
                        }
                }
                if ((long long)t == stall_ticket)
                    std::this_thread::sleep_for(std::chrono::milliseconds(stall_ms));
                else if (delay_us > 0)
                    std::this_thread::sleep_for(std::chrono::microseconds(rng() % (uint32_t)(delay_us + 1)));
                marks[k.phase][k.vol][k.unit].fetch_add(1, std::memory_order_relaxed);
                ran++;
            }
            // only a unit that ran counts: after an abort, the units of a
            // skipped unit's volume wait (and see the abort word) instead
            if (go) __atomic_fetch_add(mc_persist_done(h, q.data(), k), 1u, __ATOMIC_RELEASE);
        }
    };
    std::vector<std::thread> th;
    for (int w = 0; w < workers; ++w) th.emplace_back(worker, w);
    for (auto &x : th) x.join();
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    uint64_t dup = 0, missing = 0;
    for (int ph = 0; ph < MC_PHASES; ++ph)
        for (uint32_t v = 0; v < h.nvol; ++v)
            for (auto &m : marks[ph][v]) {
                const uint8_t c = m.load();
                if (c > 1) dup++;
                if (c == 0) missing++;
            }
    // every completion counter ends at its pass's unit count (after an
    // abort, at the units of that pass and volume that ran)
    for (int ph = 0; ph < MC_PHASES; ++ph)
        for (uint32_t v = 0; v < h.nvol; ++v) {
            uint32_t r = 0;
            for (auto &m : marks[ph][v]) r += m.load() ? 1u : 0u;
            if (q[MC_PQ_DONE + ph * h.nvol + v] != r) return 4;
            if (q[MC_PQ_ABORT] == 0 && r != mc_persist_units(h, pre, ph, v)) return 5;
        }
    printf("%u %u %llu %llu %llu %llu %.1f\n", q[MC_PQ_ABORT], q[MC_PQ_HEAD], (unsigned long long)ran.load(),
           (unsigned long long)violations.load(), (unsigned long long)dup, (unsigned long long)missing, ms);
    return 0;
}
