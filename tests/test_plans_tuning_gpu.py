"""GPU: graph plans and the autotuner give the same bits as eager calls and
as the oracle."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clean_tuning():
    cm.tuning_clear()
    yield
    cm.tuning_clear()


def test_plan_merge_replays_match_eager():
    import torch
    d = workloads.zipf(m=3_000_000, n=1_000_003)
    A, Av, B, Bv = (to_dev(d[k]) for k in ("A", "Av", "B", "Bv"))
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    plan = cm.plan_merge(A, B, Av, Bv)
    for rep in range(4):
        plan.C.zero_()
        plan.C_val.zero_()
        # eager work between replays
        Ceg, Cveg = cm.stable_merge_pairs(A, Av, B, Bv)
        torch.cuda.synchronize()
        C, Cv = plan.launch()
        torch.cuda.synchronize()
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve), f"replay {rep}"
        assert same_bits(to_host(Ceg), Ce)
    # a replay reads the inputs as they are at replay time
    d2 = workloads.zipf(seed=99, m=3_000_000, n=1_000_003)
    A.copy_(to_dev(d2["A"]))
    B.copy_(to_dev(d2["B"]))
    C, Cv = plan.launch()
    Ce2, Cve2 = oracle.stable_merge(d2["A"], d2["B"], d["Av"], d["Bv"])
    assert same_bits(to_host(C), Ce2) and same_bits(to_host(Cv), Cve2)
    plan.close()


def test_plan_keys_only_and_segmented():
    import torch
    d = workloads.segmented(seed=4, num_seg=3000, max_side=1 << 10, min_side=0)
    A, B = to_dev(d["A"]), to_dev(d["B"])
    a_off, b_off = to_dev(d["a_off"]), to_dev(d["b_off"])
    Av, Bv = to_dev(d["Av"]), to_dev(d["Bv"])
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    plan = cm.plan_segmented(A, a_off, B, b_off, Av, Bv)
    for _ in range(3):
        plan.C.zero_()
        eager = cm.stable_merge_segmented(A, a_off, B, b_off)  # eager work between replays
        torch.cuda.synchronize()
        C, Cv = plan.launch()
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
        assert same_bits(to_host(eager), Ce)
    plan.close()
    k = workloads.dup16(m=200_000, n=300_000)
    pk = cm.plan_merge(to_dev(k["A"]), to_dev(k["B"]))
    for _ in range(3):
        pk.C.zero_()
        assert same_bits(to_host(pk.launch()), oracle.stable_merge(k["A"], k["B"]))
    pk.close()


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_autotune_merge_records_and_stays_exact(dtype):
    d = workloads.dup16(m=1 << 20, n=700_001, high=1 << 12)
    A = d["A"].astype(dtype)
    B = d["B"].astype(dtype)
    best = cm.autotune_merge(to_dev(A), to_dev(B), to_dev(d["Av"]), to_dev(d["Bv"]), reps=2)
    assert 0 <= best[0] < cm.config_count() and best[1] in (0, 1) and 0 <= best[2] <= 4
    N = A.size + B.size
    assert cm.tuning_get(cm.OP_MERGE, np.dtype(dtype).name, True, N) == best
    assert cm.tuning_count() == 1
    C, Cv = cm.stable_merge_pairs(to_dev(A), to_dev(d["Av"]), to_dev(B), to_dev(d["Bv"]))
    Ce, Cve = oracle.stable_merge(A, B, d["Av"], d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


def test_autotune_segmented():
    d = workloads.segmented(seed=8, num_seg=2000, max_side=1 << 11)
    best = cm.autotune_segmented(to_dev(d["A"]), to_dev(d["a_off"]), to_dev(d["B"]),
                                 to_dev(d["b_off"]), to_dev(d["Av"]), to_dev(d["Bv"]), reps=2)
    assert best[2] == 0
    C, Cv = cm.stable_merge_segmented(to_dev(d["A"]), to_dev(d["a_off"]), to_dev(d["B"]),
                                      to_dev(d["b_off"]), to_dev(d["Av"]), to_dev(d["Bv"]))
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


def test_per_merge_launch_form_matches_batch():
    d = workloads.segmented(seed=9, num_seg=300, max_side=1 << 12, min_side=0)
    args = (to_dev(d["A"]), d["a_off"], to_dev(d["B"]), d["b_off"], to_dev(d["Av"]),
            to_dev(d["Bv"]))
    C, Cv = cm.stable_merge_segmented_each(*args)
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


def test_timing_events_per_call():
    import torch
    d = workloads.zipf(m=1_000_000, n=300_001)
    A, Av, B, Bv = (to_dev(d[k]) for k in ("A", "Av", "B", "Bv"))
    cm.timing_start(5)
    for _ in range(3):
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
    torch.cuda.synchronize()
    calls, co_rank_ms, merge_ms, starts, call_each, merge_each = cm.timing_stop(per_call=True)
    assert calls == 3 and len(call_each) == 3 and len(merge_each) == 3
    # one stream: each call starts after the previous one ended
    assert starts[0] == 0.0
    assert all(starts[c + 1] >= starts[c] + call_each[c] * 0.999 for c in range(2))
    assert co_rank_ms > 0 and merge_ms > 0
    assert all(c >= m > 0 for c, m in zip(call_each, merge_each))
    assert abs(sum(merge_each) / 3 - merge_ms) <= 1e-3 * merge_ms + 1e-6
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    # off again: a second stop is an error
    with pytest.raises(cm.CMError):
        cm.timing_stop()


def _replays_match(plan, Ce, Cve, eager, reps=3):
    import torch
    for rep in range(reps):
        plan.C.zero_()
        if plan.C_val is not None:
            plan.C_val.zero_()
        eager()  # the program's own work between replays
        torch.cuda.synchronize()
        out = plan.launch()
        torch.cuda.synchronize()
        C, Cv = out if plan.C_val is not None else (out, None)
        assert same_bits(to_host(C), Ce), f"replay {rep}: keys"
        if Cve is not None:
            assert same_bits(to_host(Cv), Cve), f"replay {rep}: payloads"


def test_plan_update_merge_same_and_new_shapes():
    """cm_plan_update_merge: other arrays of the same sizes (the executable
    graph updated in place), then sizes across the 2^24-output switch of
    the boundary pass (another kernel sequence: a new executable graph),
    then back; every replay against the oracle.  A refused update leaves
    the plan as it was."""
    import torch
    print("[plan update] merge", flush=True)
    shapes = [(40_000, 40_001, 1), (40_000, 40_001, 2), (9_000_000, 8_000_003, 3), (5, 70_000, 4)]
    plan = None
    for m, n, seed in shapes:
        d = workloads.zipf(seed=seed, m=m, n=n)
        A, Av, B, Bv = (to_dev(d[k]) for k in ("A", "Av", "B", "Bv"))
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        if plan is None:
            plan = cm.plan_merge(A, B, Av, Bv)
        else:
            plan.update(A, B, Av, Bv)
        _replays_match(plan, Ce, Cve, lambda: cm.stable_merge_pairs(A, Av, B, Bv))
    # an output over an input (checked before any capture): refused with
    # CM_EALIAS, and the plan still replays the last call
    ws = torch.empty(cm.merge_workspace_size("uint32", True, A.numel(), B.numel()),
                     dtype=torch.uint8, device=A.device)
    assert cm.load().cm_plan_update_merge(plan._handle, 0, A.data_ptr(), Av.data_ptr(), A.numel(),
                                          B.data_ptr(), Bv.data_ptr(), B.numel(), A.data_ptr(),
                                          Av.data_ptr(), ws.data_ptr(), ws.numel()) == -4
    _replays_match(plan, Ce, Cve, lambda: None, reps=1)
    # a merge plan is not a segmented plan
    assert cm.load().cm_plan_update_segmented(plan._handle, 0, None, None, None, 0, None, None,
                                              None, 0, 0, None, None, None, 0) == -1
    plan.close()


def test_plan_update_segmented():
    print("[plan update] segmented", flush=True)
    plan = None
    for seed, S in ((5, 1000), (6, 1500), (7, 1500)):
        d = workloads.segmented(seed=seed, num_seg=S, max_side=1 << 11, min_side=0)
        A, B = to_dev(d["A"]), to_dev(d["B"])
        a_off, b_off = to_dev(d["a_off"]), to_dev(d["b_off"])
        Av, Bv = to_dev(d["Av"]), to_dev(d["Bv"])
        Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                                d["Bv"])
        if plan is None:
            plan = cm.plan_segmented(A, a_off, B, b_off, Av, Bv)
        else:
            plan.update_segmented(A, a_off, B, b_off, Av, Bv)
        _replays_match(plan, Ce, Cve, lambda: cm.stable_merge_segmented(A, a_off, B, b_off))
    with pytest.raises(RuntimeError):
        plan.update(A, B, Av, Bv)
    plan.close()


def test_plan_update_across_kernel_instantiations():
    """Updates that keep the node count and types but change the kernel a
    node runs: a merge with payloads crossing 2^21 outputs (the automatic
    mode switches from the 256 x 7 to the 512 x 11 tile, one kernel either
    way), and 16-byte-aligned buffers followed by buffers 4 bytes off (the
    16-byte staging kernel, then the element-wise one), and back; every
    replay against the oracle."""
    print("[plan update] kernel instantiations", flush=True)
    cases = [((1 << 20) - 3, (1 << 20) - 5, 0), ((1 << 20) + 7, (1 << 20) + 1, 0),
             ((1 << 20) + 7, (1 << 20) + 1, 1), (600_001, 500_003, 1), (600_001, 500_003, 0)]
    plan = None
    for seed, (m, n, off) in enumerate(cases):
        d = workloads.dup16(seed=50 + seed, m=m, n=n)
        A, Av, B, Bv = (to_dev(d[k], off) for k in ("A", "Av", "B", "Bv"))
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        if plan is None:
            plan = cm.plan_merge(A, B, Av, Bv)
        else:
            plan.update(A, B, Av, Bv)
        _replays_match(plan, Ce, Cve, lambda: cm.stable_merge_pairs(A, Av, B, Bv))
    plan.close()
    # keys only, aligned then not
    plan = None
    for seed, off in enumerate((0, 1, 0)):
        d = workloads.dup16(seed=70 + seed, m=300_001, n=200_002)
        A, B = to_dev(d["A"], off), to_dev(d["B"], off)
        Ce, _ = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        if plan is None:
            plan = cm.plan_merge(A, B)
        else:
            plan.update(A, B)
        _replays_match(plan, Ce, None, lambda: cm.stable_merge(A, B))
    plan.close()
