"""GPU parity at the full workload sizes, element by element against the
oracle (which merges 3e8 elements in well under a second), in the default
launch configuration and, for the headline merge and the segmented batch,
in the one bench.py times (the autotuner's choice on the same arrays).

- single uneven merge: m = 2^28, n = 2^26, uint32 Zipf keys + payloads;
- m = n = 2^27: uint64 uniform keys, float32 N(0,1) keys, and the three
  structured uint32 cases (A below B, interleaved, all equal);
- 65,536 independent merges, sides log-uniform in [1, 2^16].
Each test prints its case before touching the GPU."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def run_and_compare(name, d):
    import torch
    print(f"[full-size] {name}: m={d['A'].size} n={d['B'].size} {d['A'].dtype}", flush=True)
    C, Cv = cm.stable_merge_pairs(to_dev(d["A"]), to_dev(d["Av"]), to_dev(d["B"]), to_dev(d["Bv"]))
    C, Cv = to_host(C), to_host(Cv)
    torch.cuda.empty_cache()
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    assert same_bits(C, Ce), f"{name}: keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"{name}: payloads differ first at {first_difference(Cv, Cve)}"


def test_zipf_uneven_full():
    run_and_compare("zipf 2^28 + 2^26", workloads.zipf())


def test_u64_full():
    run_and_compare("uint64 2^27 + 2^27", workloads.u64())


def test_f32_full():
    run_and_compare("float32 2^27 + 2^27", workloads.f32())


@pytest.mark.parametrize("kind", ["a_below_b", "interleaved", "all_equal"])
def test_structured_full(kind):
    run_and_compare(f"{kind} 2^27 + 2^27", workloads.structured(kind))


def test_segmented_batch_full():
    import torch
    d = workloads.segmented()
    print(f"[full-size] segmented: {d['a_off'].size - 1} segments, "
          f"{d['A'].size + d['B'].size} outputs", flush=True)
    C, Cv = cm.stable_merge_segmented(to_dev(d["A"]), to_dev(d["a_off"]), to_dev(d["B"]),
                                      to_dev(d["b_off"]), to_dev(d["Av"]), to_dev(d["Bv"]))
    C, Cv = to_host(C), to_host(Cv)
    torch.cuda.empty_cache()
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"


def test_zipf_autotuned_full():
    """The headline merge in the configuration the autotuner picks (as
    bench.py does before timing), then compared to the oracle."""
    import torch
    d = workloads.zipf()
    print(f"[full-size] zipf autotuned: m={d['A'].size} n={d['B'].size}", flush=True)
    A, B, Av, Bv = (to_dev(d[k]) for k in ("A", "B", "Av", "Bv"))
    try:
        choice = cm.autotune_merge(A, B, Av, Bv, reps=1)
        print(f"[full-size] tuned choice {choice}", flush=True)
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
        C, Cv = to_host(C), to_host(Cv)
    finally:
        cm.tuning_clear()
    del A, B, Av, Bv
    torch.cuda.empty_cache()
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"


def test_segmented_autotuned_full():
    import torch
    d = workloads.segmented()
    print(f"[full-size] segmented autotuned: {d['a_off'].size - 1} segments", flush=True)
    A, B, Av, Bv = (to_dev(d[k]) for k in ("A", "B", "Av", "Bv"))
    ao, bo = to_dev(d["a_off"]), to_dev(d["b_off"])
    try:
        choice = cm.autotune_segmented(A, ao, B, bo, Av, Bv, reps=1)
        print(f"[full-size] tuned choice {choice}", flush=True)
        C, Cv = cm.stable_merge_segmented(A, ao, B, bo, Av, Bv)
        C, Cv = to_host(C), to_host(Cv)
    finally:
        cm.tuning_clear()
    del A, B, Av, Bv
    torch.cuda.empty_cache()
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"],
                                            d["Bv"])
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"
