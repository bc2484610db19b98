"""Host checks of the PyTorch entry points: a plan, output or workspace that
does not match the input is rejected before any pointer reaches the C ABI
(the library sees raw pointers only and would read or write past them)."""
import pytest
import torch

from paper_1906_11355_amd import api
from paper_1906_11355_amd._lib import Plan


def _plan(shape=(16, 20), dtype="float32", out="float32"):
    return Plan(shape, (4, 5), 32, 0.02, in_dtype=dtype, out_dtype=out)


def test_matching_tensors_pass():
    p = _plan()
    x = torch.zeros(16, 20)
    api._check_against_plan(p, x, torch.zeros(16, 20))
    api._check_workspace(torch.zeros(p.workspace_size(), dtype=torch.uint8), p.workspace_size(), x.device)


@pytest.mark.parametrize("x,out,msg", [
    (torch.zeros(16, 21), None, "input shape"),
    (torch.zeros(32, 20), None, "input shape"),
    (torch.zeros(16, 20, dtype=torch.uint8), None, "input dtype"),
    (torch.zeros(16, 20), torch.zeros(16, 19), "output shape"),
    (torch.zeros(16, 20), torch.zeros(16, 20, dtype=torch.uint8), "output dtype"),
])
def test_mismatch_is_rejected(x, out, msg):
    with pytest.raises(ValueError, match=msg):
        api._check_against_plan(_plan(), x, out)


def test_integer_output_plan_needs_integer_output():
    p = _plan(dtype="uint16", out="uint16")
    api._check_against_plan(p, torch.zeros(16, 20, dtype=torch.uint16), torch.zeros(16, 20, dtype=torch.uint16))
    with pytest.raises(ValueError, match="output dtype"):
        api._check_against_plan(p, torch.zeros(16, 20, dtype=torch.uint16), torch.zeros(16, 20))


def test_small_workspace_is_rejected():
    p = _plan()
    need = p.workspace_size()
    with pytest.raises(ValueError, match="needed"):
        api._check_workspace(torch.zeros(need - 1, dtype=torch.uint8), need, torch.device("cpu"))
    # bytes count, not elements
    api._check_workspace(torch.zeros((need + 3) // 4, dtype=torch.float32), need, torch.device("cpu"))
