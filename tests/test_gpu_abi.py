"""GPU checks of the C ABI's failure paths: a device workspace allocation that
fails while a plan is built comes back as FSI_ERR_OUT_OF_MEMORY and frees
everything already allocated; plans are destroyed while their work runs."""
import numpy as np
import pytest
import torch

from paper_2601_01903_amd import BatchPlan, FsiError, Plan

pytestmark = pytest.mark.gpu


def test_device_allocation_failure_frees_everything(monkeypatch):
    torch.cuda.synchronize()
    # a first plan warms up the runtime's own allocations
    BatchPlan([20] * 8, [4] * 8, dtype="f32").close()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    monkeypatch.setenv("FSI_TEST_FAIL_ALLOC", "device")
    for _ in range(3):
        with pytest.raises(FsiError) as ei:
            BatchPlan([20] * 8, [4] * 8, dtype="f32")
        assert ei.value.status == 3
    with pytest.raises(FsiError):
        Plan(16, 3, dtype="f32")
    monkeypatch.delenv("FSI_TEST_FAIL_ALLOC")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    # each failed plan had tables and per-tile buffers of tens of MB on the
    # device before its workspace allocation failed
    print(f"free before {free0 >> 20} MiB, after {free1 >> 20} MiB", flush=True)
    assert free0 - free1 < (16 << 20)
    # and plans still build and run afterwards
    bp = BatchPlan([12], [3], dtype="f32")
    out = bp.apply(torch.zeros(1 << 12, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    bp.close()


def test_destroy_waits_for_plan_work_only():
    """Destroying a plan right after an apply returns correct outputs (the
    plan's event is waited on) and leaves other streams' work alone."""
    x = torch.randn(1 << 20, dtype=torch.float32, device="cuda")
    ref_plan = BatchPlan([20], [4], dtype="f32")
    ref = ref_plan.apply(x, graph=False)
    torch.cuda.synchronize()
    ref_plan.close()
    for graph in (False, True):
        bp = BatchPlan([20], [4], dtype="f32")
        out = bp.apply(x, graph=graph)
        bp.close()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_graph_pointer_change_updates_in_place():
    """A batched apply with a new (values, out) pair updates the captured
    graph's arguments; every pointer pair gives its own correct result."""
    bp = BatchPlan([16, 12], [3, 4], dtype="f32")
    xs = [torch.randn(bp.value_offset[-1], dtype=torch.float32, device="cuda") for _ in range(3)]
    refs = [bp.apply(x, graph=False) for x in xs]
    outs = [torch.empty_like(r) for r in refs]
    for rep in range(2):
        for x, o in zip(xs, outs):
            bp.apply(x, o, graph=True)
        torch.cuda.synchronize()
        for r, o in zip(refs, outs):
            assert torch.equal(r, o)
    bp.close()
