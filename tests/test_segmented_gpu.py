"""GPU parity of the segmented batch against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("restore_settings")]


def run_seg(d, payload=True):
    args = dict(A_val=to_dev(d["Av"]), B_val=to_dev(d["Bv"])) if payload else {}
    out = cm.stable_merge_segmented(to_dev(d["A"]), to_dev(d["a_off"]), to_dev(d["B"]),
                                    to_dev(d["b_off"]), **args)
    if payload:
        return to_host(out[0]), to_host(out[1])
    return to_host(out), None


def check_seg(d, payload=True):
    C, Cv = run_seg(d, payload)
    if payload:
        Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"],
                                                d["Av"], d["Bv"])
        assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"
    else:
        Ce = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"])
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"


def as_dtype(d, dtype):
    d = dict(d)
    if np.dtype(dtype) == np.float32:
        d["A"] = d["A"].astype(np.float32) - 512.0
        d["B"] = d["B"].astype(np.float32) - 512.0
    else:
        d["A"] = d["A"].astype(dtype)
        d["B"] = d["B"].astype(dtype)
    return d


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_many_tiny_segments_with_empty_sides(dtype):
    d = as_dtype(workloads.segmented(seed=5, num_seg=5000, max_side=40, key_high=16, min_side=0),
                 dtype)
    check_seg(d)
    check_seg(d, payload=False)


@pytest.mark.parametrize("search,partition,stride", [(0, 0, 64), (1, 0, 64), (0, 2, 64), (1, 2, 64),
                                                     (1, 2, 16)])
def test_all_configs(search, partition, stride):
    cm.set_search(search)
    cm.set_partition(partition)
    cm.set_coarse_stride(stride)
    d = workloads.segmented(seed=7, num_seg=700, max_side=1 << 12, key_high=64, min_side=0)
    for c in range(cm.config_count()):
        cm.set_config("uint32", True, c)
        cm.set_config("uint32", False, c)
        check_seg(d)
        check_seg(d, payload=False)


def test_single_segment_equals_plain_merge():
    d = workloads.dup16(m=100_000, n=77_777, high=300)
    d["a_off"] = np.array([0, d["A"].size], dtype=np.uint64)
    d["b_off"] = np.array([0, d["B"].size], dtype=np.uint64)
    C, Cv = run_seg(d)
    C2, Cv2 = cm.stable_merge_pairs(to_dev(d["A"]), to_dev(d["Av"]), to_dev(d["B"]),
                                    to_dev(d["Bv"]))
    assert same_bits(C, to_host(C2)) and same_bits(Cv, to_host(Cv2))


def test_edge_layouts():
    """All-empty segments, segments empty on one side, empty at both ends."""
    rng = np.random.default_rng(12)
    la = np.array([0, 0, 5, 0, 3000, 0, 1, 0, 0], dtype=np.int64)
    lb = np.array([0, 4, 0, 0, 1, 2500, 1, 7, 0], dtype=np.int64)
    A = np.concatenate([np.sort(rng.integers(0, 9, x)) for x in la]).astype(np.uint32)
    B = np.concatenate([np.sort(rng.integers(0, 9, x)) for x in lb]).astype(np.uint32)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    check_seg(dict(A=A, B=B, a_off=a_off, b_off=b_off, Av=Av, Bv=Bv))
    # every segment empty
    z = np.zeros(0, dtype=np.uint32)
    zo = np.zeros(4, dtype=np.uint64)
    C = cm.stable_merge_segmented(to_dev(np.zeros(1, np.uint32))[:0], to_dev(zo), to_dev(z),
                                  to_dev(zo))
    assert C.numel() == 0


def test_inconsistent_offsets_leave_output_untouched():
    """Offsets that do not end at the array lengths are refused on the device
    (flag set, nothing written, no access outside the arrays)."""
    import torch
    d = workloads.segmented(seed=3, num_seg=50, max_side=100)
    a_off = d["a_off"].copy()
    a_off[-1] -= 1
    C = torch.full((d["A"].size + d["B"].size,), 7, dtype=torch.uint32, device="cuda:0")
    cm.stable_merge_segmented(to_dev(d["A"]), to_dev(a_off), to_dev(d["B"]), to_dev(d["b_off"]),
                              C=C)
    assert np.all(to_host(C) == 7)
    a_off = d["a_off"].copy()
    a_off[10], a_off[11] = a_off[11], a_off[10]  # not monotone
    cm.stable_merge_segmented(to_dev(d["A"]), to_dev(a_off), to_dev(d["B"]), to_dev(d["b_off"]),
                              C=C)
    assert np.all(to_host(C) == 7)


@pytest.mark.parametrize("partition", [0, 2])
def test_two_level_segmented_edges(partition):
    """Many blocks and coarse windows spanning many tiny segments, empty
    segments, and segments much longer than a coarse window."""
    cm.set_partition(partition)
    cm.set_coarse_stride(16)
    rng = np.random.default_rng(44)
    la = np.concatenate([rng.integers(0, 3, 3000), [200_000], rng.integers(0, 50, 2000), [0, 0],
                         [90_001]]).astype(np.int64)
    lb = np.concatenate([rng.integers(0, 3, 3000), [3], rng.integers(0, 50, 2000), [0, 7],
                         [150_000]]).astype(np.int64)
    A = np.concatenate([np.sort(rng.integers(0, 5, x)) for x in la]).astype(np.uint32)
    B = np.concatenate([np.sort(rng.integers(0, 5, x)) for x in lb]).astype(np.uint32)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    check_seg(dict(A=A, B=B, a_off=a_off, b_off=b_off, Av=Av, Bv=Bv))


def test_reduced_batch_workload():
    """The batch recipe (log-uniform sides, keys uniform in [0, 2**20)) at
    4096 segments of up to 2**12 per side."""
    d = workloads.segmented(num_seg=4096, max_side=1 << 12)
    check_seg(d)


@pytest.mark.parametrize("offset", [1, 2])
def test_misaligned_bases_segmented(offset):
    """Bases off 16-byte alignment take the element-wise staging path."""
    d = workloads.segmented(seed=19, num_seg=900, max_side=1 << 11, min_side=0)
    C, Cv = cm.stable_merge_segmented(to_dev(d["A"], offset), to_dev(d["a_off"]),
                                      to_dev(d["B"], offset), to_dev(d["b_off"]),
                                      to_dev(d["Av"], offset), to_dev(d["Bv"], offset))
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    for dtype in (np.uint64, np.float32):
        e = as_dtype(d, dtype)
        C = cm.stable_merge_segmented(to_dev(e["A"], offset), to_dev(e["a_off"]),
                                      to_dev(e["B"], offset), to_dev(e["b_off"]))
        assert same_bits(to_host(C), oracle.stable_merge_segmented(e["A"], e["a_off"], e["B"],
                                                                   e["b_off"]))
