"""C ABI checks that need no GPU.

- the shared library loads and exports every function include/*.h declares;
- cm_co_rank_host (the library's own CPU Algorithm 1) equals the oracle;
- argument errors are reported synchronously, before anything would be
  launched (these calls pass made-up addresses that are never touched).
"""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

OK, EINVAL, ERANGE, EDTYPE, EALIAS, ENOSPC, ECONFIG = 0, -1, -2, -3, -4, -5, -8


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(cm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cm_co_rank", "cm_co_rank_host", "cm_stable_merge", "cm_stable_merge_pairs",
                     "cm_stable_merge_segmented"):
        assert required in names


def test_library_exports_every_declared_function():
    lib = cm.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(cm.EXPORTS)


def test_status_strings_and_version():
    assert cm.load().cm_version() >= 1
    assert cm.status_string(OK) == "ok"
    assert cm.status_string(ENOSPC) == "workspace or arena too small"


def test_host_co_rank_figure(figure):
    A = np.array(figure["A"]["keys"], dtype=np.uint32)
    B = np.array(figure["B"]["keys"], dtype=np.uint32)
    assert cm.co_rank_host(22, A, B) == (12, 10)
    for i in range(A.size + B.size + 1):
        assert cm.co_rank_host(i, A, B) == oracle.co_rank_brute(i, A, B)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_host_co_rank_random(dtype):
    rng = np.random.default_rng(5)
    for m, n, hi in ((0, 0, 3), (0, 7, 3), (9, 0, 3), (500, 1500, 20), (4096, 4000, 2)):
        A = np.sort(rng.integers(0, hi, m)).astype(dtype)
        B = np.sort(rng.integers(0, hi, n)).astype(dtype)
        for i in sorted(set(rng.integers(0, m + n + 1, 40).tolist()) | {0, m + n}):
            assert cm.co_rank_host(i, A, B) == oracle.co_rank_brute(i, A, B)


def test_host_co_rank_errors():
    A = np.zeros(3, dtype=np.uint32)
    with pytest.raises(cm.CMError) as e:
        cm.co_rank_host(7, A, A)
    assert e.value.status == ERANGE
    lib = cm.load()
    j, k = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.cm_co_rank_host(9, 0, None, 0, None, 0, ctypes.byref(j), ctypes.byref(k)) == EDTYPE
    assert lib.cm_co_rank_host(0, 0, None, 4, None, 0, ctypes.byref(j), ctypes.byref(k)) == EINVAL


def test_merge_argument_errors_are_synchronous():
    lib = cm.load()
    P = ctypes.c_void_p
    A, B, C = P(0x10000000), P(0x20000000), P(0x30000000)
    ws = P(0x40000000)
    big = 1 << 20
    # unknown key type
    assert lib.cm_stable_merge(9, A, 4, B, 4, C, ws, big, None) == EDTYPE
    # null with nonzero length
    assert lib.cm_stable_merge(0, None, 4, B, 4, C, ws, big, None) == EINVAL
    assert lib.cm_stable_merge_pairs(0, A, None, 4, B, P(0x50000000), 4, C, P(0x60000000),
                                     ws, big, None) == EINVAL
    # output overlapping an input
    assert lib.cm_stable_merge(0, A, 4, B, 4, P(0x10000000 + 8), ws, big, None) == EALIAS
    assert lib.cm_stable_merge_pairs(0, A, P(0x50000000), 4, B, P(0x60000000), 4, C,
                                     P(0x50000000), ws, big, None) == EALIAS
    # 8-byte payloads: overlaps are judged on 8-byte elements (C_val 24 bytes
    # into A_val's 32 overlaps)
    assert lib.cm_stable_merge_pairs64(0, A, None, 4, B, P(0x60000000), 4, C, P(0x70000000),
                                       ws, big, None) == EINVAL
    assert lib.cm_stable_merge_pairs64(0, A, P(0x50000000), 4, B, P(0x60000000), 4, C,
                                       P(0x50000000 + 24), ws, big, None) == EALIAS
    assert lib.cm_stable_merge_pairs64(9, A, P(0x50000000), 4, B, P(0x60000000), 4, C,
                                       P(0x70000000), ws, big, None) == EDTYPE
    assert lib.cm_stable_merge_pairs64(0, None, None, 0, None, None, 0, None, None, None, 0,
                                       None) == OK
    # workspace too small
    need = lib.cm_merge_workspace_size(0, 0, 1 << 20, 1 << 20)
    assert need > 0
    assert lib.cm_stable_merge(0, A, 1 << 20, B, 1 << 20, C, ws, need - 1, None) == ENOSPC
    assert lib.cm_stable_merge(0, A, 1 << 20, B, 1 << 20, C, None, 0, None) == ENOSPC
    # empty merge is a no-op
    assert lib.cm_stable_merge(0, None, 0, None, 0, None, None, 0, None) == OK
    # segmented
    assert lib.cm_stable_merge_segmented(0, None, None, None, 0, None, None, None, 0, 0, None,
                                         None, None, 0, None) == OK
    assert lib.cm_stable_merge_segmented(0, A, None, None, 4, B, None, None, 4, 0, C, None, ws,
                                         big, None) == EINVAL
    assert lib.cm_stable_merge_segmented(0, A, None, P(0x70000000), 4, B, None, P(0x71000000), 4,
                                         1 << 32, C, None, ws, big, None) == EINVAL
    # arrays of 2^48 elements or more (byte counts would wrap), even with room
    huge = 1 << 48
    assert lib.cm_stable_merge(0, A, huge, B, 4, C, ws, big, None) == EINVAL
    assert lib.cm_stable_merge(0, A, 4, B, (1 << 64) - 1, C, ws, big, None) == EINVAL
    assert lib.cm_stable_merge_segmented(0, A, None, P(0x70000000), huge, B, None, P(0x71000000),
                                         4, 1, C, None, ws, big, None) == EINVAL
    assert lib.cm_co_rank(0, P(0x80000000), 1, A, huge, B, 4, P(0x90000000), None) == EINVAL
    assert lib.cm_stable_sort(0, A, huge, C, ws, big, None) == EINVAL
    # co_rank on device arrays
    assert lib.cm_co_rank(0, None, 3, A, 4, B, 4, P(0x80000000), None) == EINVAL
    assert lib.cm_co_rank(0, P(0x80000000), 4, A, 4, B, 4, P(0x80000000 + 8), None) == EALIAS


def test_config_table(restore_settings):
    n = cm.config_count()
    assert n >= 4
    tiles = set()
    for c in range(n):
        nt, e = cm.config_info(c)
        assert nt % 64 == 0 and e % 2 == 1
        tiles.add(nt * e)
    assert len(tiles) == n
    with pytest.raises(cm.CMError):
        cm.config_info(n)
    old = cm.get_config("uint32", True)
    cm.set_config("uint32", True, n - 1)
    assert cm.get_config("uint32", True) == n - 1
    cm.set_config("uint32", True, old)
    assert cm.load().cm_set_config(0, 1, n) == ECONFIG
    assert cm.load().cm_set_config(0, 1, -2) == ECONFIG
    assert cm.load().cm_set_search(2) == EINVAL
    # block order: workgroup order, one run per XCD, or runs of up to 2^20 blocks
    for order in (0, 1, 2, 32, 1 << 20):
        assert cm.load().cm_set_block_order(order) == OK
        assert cm.get_block_order() == order
    assert cm.load().cm_set_block_order(-1) == EINVAL
    assert cm.load().cm_set_block_order((1 << 20) + 1) == EINVAL
    for mode in range(-1, 5):
        cm.set_partition(mode)
        assert cm.get_partition() == mode
    assert cm.load().cm_set_partition(5) == EINVAL
    assert cm.load().cm_set_fine_lanes(3) == EINVAL and cm.load().cm_set_fine_lanes(8) == EINVAL
    assert cm.load().cm_set_partition(-2) == EINVAL
    assert cm.load().cm_tuning_set(0, 0, 1, 20, 0, 1, 5) == EINVAL


def test_workspace_sizes(restore_settings):
    lib = cm.load()
    for c in range(cm.config_count()):
        cm.set_config("uint32", False, c)
        nt, e = cm.config_info(c)
        T = nt * e
        for N in (1, T - 1, T, T + 1, 10 * T + 3):
            tiles = -(-N // T)
            assert lib.cm_merge_workspace_size(0, 0, N, 0) >= 8 * (tiles + 1)
            assert lib.cm_merge_workspace_size(0, 0, N, 0) % 256 == 0
    assert lib.cm_merge_workspace_size(0, 0, 0, 0) == 0


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(cm, "_lib", None)
    monkeypatch.setattr(cm, "library_path", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        cm.load()


def test_workloads_shapes():
    d = workloads.zipf(m=1 << 16, n=1 << 14)
    assert d["A"].dtype == np.uint32 and d["A"].size == 1 << 16
    assert np.all(np.diff(d["A"].astype(np.int64)) >= 0)
    assert len(np.unique(np.concatenate([d["A"], d["B"]]))) <= 1024
    s = workloads.segmented(num_seg=64, max_side=1 << 10)
    assert s["a_off"][-1] == s["A"].size and s["b_off"][-1] == s["B"].size
    assert np.all(np.diff(s["a_off"].astype(np.int64)) >= 1)


def test_tuning_table_host_logic(tmp_path, restore_settings):
    """The tuning table is host state: set / get / save / load / clear."""
    cm.set_partition(-1)
    cm.set_config("uint32", True, -1)
    cm.set_config("uint32", False, -1)
    cm.tuning_clear()
    assert cm.tuning_count() == 0
    default = cm.tuning_get(cm.OP_MERGE, "uint32", True, 1000)
    # automatic boundary pass: none below 2^24 outputs, two-level from
    # there and for batches; no configuration set: the per-operation tiles
    assert cm.get_partition() == -1
    assert cm.get_config("uint32", True) == -1 and cm.get_config("uint32", False) == -1
    assert default == (0, cm.get_search(), 4)
    assert cm.tuning_get(cm.OP_MERGE, "uint32", True, (1 << 24) - 1)[2] == 4
    assert cm.tuning_get(cm.OP_MERGE, "uint32", True, 1 << 24)[2] == 2
    assert cm.tuning_get(cm.OP_MERGE, "uint32", False, (1 << 24) - 1)[2] == 4
    assert cm.tuning_get(cm.OP_MERGE, "uint32", False, 1 << 24)[2] == 2
    # tiles: 256 x 7 with payloads, 256 x 9 keys only; 512 x 11 where the
    # pass is skipped from 2^21 outputs (2^22 keys only)
    tile = lambda v, N: cm.tuning_get(cm.OP_MERGE, "uint32", v, N)[0]
    assert [tile(True, N) for N in (1 << 20, (1 << 21) - 1, 1 << 21, 1 << 23, 1 << 24)] == [0, 0, 7, 7, 0]
    assert [tile(False, N) for N in (1 << 21, (1 << 22) - 1, 1 << 22, 1 << 23, 1 << 24)] == [6, 6, 7, 7, 6]
    assert cm.tuning_get(cm.OP_SEGMENTED, "uint32", True, 1 << 20)[0] == 2
    assert cm.tuning_get(cm.OP_BATCH, "uint32", True, 1 << 20)[0] == 2
    # a set configuration wins over every default, and -1 unsets it
    cm.set_config("uint32", False, 3)
    assert tile(False, 1 << 22) == 3 and tile(False, 1 << 24) == 3
    cm.set_config("uint32", False, -1)
    assert cm.get_config("uint32", False) == -1 and tile(False, 1 << 22) == 7
    assert cm.tuning_get(cm.OP_SEGMENTED, "uint32", True, 1000)[2] == 2
    # a batch of separate merges: two-level pass automatically, any mode
    # when set, the streaming mode taken as two-level
    assert cm.tuning_get(cm.OP_BATCH, "uint32", True, 1 << 30)[2] == 2
    for mode, batch_mode in ((0, 0), (1, 1), (2, 2), (3, 2), (4, 4)):
        cm.set_partition(mode)
        assert cm.tuning_get(cm.OP_BATCH, "uint32", True, 1 << 20)[2] == batch_mode
    cm.set_partition(-1)
    with pytest.raises(cm.CMError):
        cm.tuning_get(cm.OP_SORT + 1, "uint32", True, 1000)
    with pytest.raises(cm.CMError):
        cm.tuning_get(-1, "uint32", True, 1000)
    cm.tuning_set(cm.OP_MERGE, "uint32", True, 10, 3, 0, 0)  # size class 10: N in [512, 1024)
    assert cm.tuning_get(cm.OP_MERGE, "uint32", True, 1000) == (3, 0, 0)
    assert cm.tuning_get(cm.OP_MERGE, "uint32", True, 1024) == default
    assert cm.tuning_get(cm.OP_MERGE, "uint32", False, 1000) == (6, cm.get_search(), 4)
    cm.tuning_set(cm.OP_SEGMENTED, "uint64", False, 30, 5, 1, 0)
    path = tmp_path / "tune.txt"
    cm.tuning_save(str(path))
    assert len([l for l in path.read_text().splitlines() if not l.startswith("#")]) == 2
    cm.tuning_clear()
    assert cm.tuning_count() == 0
    cm.tuning_load(str(path))
    assert cm.tuning_count() == 2
    assert cm.tuning_get(cm.OP_SEGMENTED, "uint64", False, 1 << 29) == (5, 1, 0)
    bad = tmp_path / "bad.txt"
    bad.write_text("0 0 1 10 99 0 0 1.0\n")
    with pytest.raises(cm.CMError):
        cm.tuning_load(str(bad))
    assert cm.tuning_count() == 2
    with pytest.raises(cm.CMError):
        cm.tuning_set(cm.OP_MERGE, "uint32", True, 10, cm.config_count(), 0, 0)
    cm.tuning_clear()


def test_tuning_file_identity(tmp_path, monkeypatch):
    """A saved table names the device architecture, HIP runtime and library
    build it was timed with; one naming anything else, or nothing, is
    refused with CM_ESTALE and leaves the table as it was.  With no path the
    file is $CM_TUNING_FILE, else the user's cache directory."""
    cm.tuning_clear()
    cm.tuning_set(cm.OP_MERGE, "uint32", True, 12, 2, 1, 0)
    good = tmp_path / "tune.txt"
    cm.tuning_save(str(good))
    text = good.read_text()
    head = [l for l in text.splitlines() if l.startswith("#")]
    assert head[0] == "# corank_merge tuning v2"
    assert f"# library {cm.build_id()}" in head
    assert any(l.startswith("# arch ") for l in head) and any(l.startswith("# hip_runtime ") for l in head)
    assert len(cm.build_id()) == 16
    cm.tuning_clear()
    cm.tuning_load(str(good))
    assert cm.tuning_count() == 1
    for old, new in (("# library " + cm.build_id(), "# library 0123456789abcdef"),
                     ("# arch ", "# arch gfx000-"), ("# hip_runtime ", "# hip_runtime 1")):
        stale = tmp_path / "stale.txt"
        line = next(l for l in text.splitlines() if l.startswith(old))
        stale.write_text(text.replace(line, line.replace(old, new) if old.endswith(" ") else new))
        cm.tuning_clear()
        with pytest.raises(cm.CMError) as err:
            cm.tuning_load(str(stale))
        assert err.value.status == cm.ESTALE
        assert cm.tuning_count() == 0
    # an identity-free table (the old format) is refused the same way
    plain = tmp_path / "plain.txt"
    plain.write_text("\n".join(l for l in text.splitlines() if not l.startswith("#")) + "\n")
    with pytest.raises(cm.CMError) as err:
        cm.tuning_load(str(plain))
    assert err.value.status == cm.ESTALE
    # default location: the environment variable, then the cache directory
    env_file = tmp_path / "env" / "t.txt"
    env_file.parent.mkdir()
    monkeypatch.setenv("CM_TUNING_FILE", str(env_file))
    cm.tuning_set(cm.OP_MERGE, "uint32", True, 12, 2, 1, 0)
    cm.tuning_save()
    assert env_file.read_text() == text
    cm.tuning_clear()
    cm.tuning_load()
    assert cm.tuning_get(cm.OP_MERGE, "uint32", True, 3000)[:3] == (2, 1, 0)
    monkeypatch.delenv("CM_TUNING_FILE")
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path / "cache"))
    cm.tuning_save()
    assert (tmp_path / "cache" / "corank_merge" / "tuning.txt").read_text() == text
    cm.tuning_clear()


def test_plan_and_tuner_argument_errors():
    lib = cm.load()
    P = ctypes.c_void_p
    h = ctypes.c_void_p()
    assert lib.cm_plan_create_merge(9, None, None, 0, None, None, 0, None, None, None, 0,
                                    ctypes.byref(h)) == EDTYPE
    assert h.value is None
    assert lib.cm_plan_create_merge(0, None, None, 5, None, None, 0, P(0x1000), None, P(0x2000),
                                    1 << 20, ctypes.byref(h)) == EINVAL
    assert lib.cm_plan_launch(None, None) == EINVAL
    assert lib.cm_plan_update_merge(None, 0, None, None, 0, None, None, 0, None, None, None,
                                    0) == EINVAL
    assert lib.cm_plan_update_segmented(None, 0, None, None, None, 0, None, None, None, 0, 0,
                                        None, None, None, 0) == EINVAL
    assert lib.cm_plan_destroy(None) == EINVAL
    best = (ctypes.c_int * 3)()
    assert lib.cm_autotune_merge(0, P(0x1000), None, 4, P(0x2000), None, 4, P(0x3000), None,
                                 P(0x4000), 1 << 20, 0, None, best) == EINVAL
    assert lib.cm_autotune_merge(0, None, None, 0, None, None, 0, None, None, None, 0, 3, None,
                                 best) == EINVAL


def test_batch_prepare_and_argument_errors():
    """cm_batch_prepare is host-only; bad batch arguments fail before launch."""
    import numpy as np
    lib = cm.load()
    fields = ("A", "A_val", "m", "B", "B_val", "n", "C", "C_val", "first_block")
    descs = np.zeros(3, dtype=np.dtype([(f, np.uint64) for f in fields]))
    sizes = [(5000, 7000), (0, 0), (1, 1 << 20)]
    base = 1 << 32
    for r, (m, n) in enumerate(sizes):
        descs[r] = (base + r * (1 << 28), 0, m, base + r * (1 << 28) + (1 << 26), 0, n,
                    base + r * (1 << 28) + (1 << 27), 0, 0)
    total = ctypes.c_uint64()
    assert lib.cm_batch_prepare(0, 0, descs.ctypes.data_as(ctypes.c_void_p), 3,
                                ctypes.byref(total)) == OK
    cfg, _, _ = cm.tuning_get(cm.OP_BATCH, "uint32", False, sum(m + n for m, n in sizes))
    nt, e = cm.config_info(cfg)
    T = nt * e
    expect = [-(-(m + n) // T) for m, n in sizes]
    assert descs["first_block"].tolist() == [0, expect[0], expect[0] + expect[1]]
    assert total.value == sum(expect)
    P = ctypes.c_void_p
    need = lib.cm_batch_workspace_size(total.value, 3)
    dp = descs.ctypes.data_as(ctypes.c_void_p)
    # first_block that does not match the block size
    bad = descs.copy()
    bad["first_block"][2] += 1
    assert lib.cm_stable_merge_batch(0, 0, bad.ctypes.data_as(ctypes.c_void_p), P(0x1000), 3,
                                     total.value, P(0x2000), need, None) == EINVAL
    # workspace too small
    assert lib.cm_stable_merge_batch(0, 0, dp, P(0x1000), 3, total.value, P(0x2000), need - 8,
                                     None) == ENOSPC
    # output of merge 2 overlapping the input of merge 0
    alias = descs.copy()
    alias["C"][2] = alias["A"][0] + 16
    assert lib.cm_stable_merge_batch(0, 0, alias.ctypes.data_as(ctypes.c_void_p), P(0x1000), 3,
                                     total.value, P(0x2000), need, None) == EALIAS
    # two outputs overlapping each other
    alias = descs.copy()
    alias["C"][2] = alias["C"][0] + 64
    assert lib.cm_stable_merge_batch(0, 0, alias.ctypes.data_as(ctypes.c_void_p), P(0x1000), 3,
                                     total.value, P(0x2000), need, None) == EALIAS
    # payload pointer given in a keys-only batch
    pay = descs.copy()
    pay["A_val"][0] = 0x5000
    assert lib.cm_stable_merge_batch(0, 0, pay.ctypes.data_as(ctypes.c_void_p), P(0x1000), 3,
                                     total.value, P(0x2000), need, None) == EINVAL
    assert lib.cm_stable_merge_batch(0, 0, None, None, 0, 0, None, 0, None) == OK
    # no device copy of the descriptors: allowed up to CM_BATCH_INLINE_MAX
    # merges (checked here with an output over an input, refused before any
    # launch), refused above
    assert lib.cm_stable_merge_batch(0, 0, alias.ctypes.data_as(ctypes.c_void_p), None, 3,
                                     total.value, P(0x2000), need, None) == EALIAS
    over = np.zeros(cm.BATCH_INLINE_MAX + 1, dtype=descs.dtype)
    assert lib.cm_batch_prepare(0, 0, over.ctypes.data_as(ctypes.c_void_p), len(over),
                                ctypes.byref(total)) == OK
    assert lib.cm_stable_merge_batch(0, 0, over.ctypes.data_as(ctypes.c_void_p), None, len(over),
                                     total.value, P(0x2000), 1 << 20, None) == EINVAL
    # the workspace holds one co-rank per block end and a coarse part
    assert lib.cm_batch_workspace_size(1000, 24) >= 8 * 1024 + 8 * (1024 // 16) + 4 * 1000
    # a batch whose block count reaches 2^31 is refused (checked merge by
    # merge, so the running sum cannot wrap); one such merge alone is fine
    many = np.zeros(64, dtype=descs.dtype)
    for r in range(64):
        many[r] = (base + r * (1 << 44), 0, (1 << 40) - 1, base + r * (1 << 44) + (1 << 43), 0,
                   1, base + r * (1 << 44) + (3 << 42), 0, 0)
    assert lib.cm_batch_prepare(0, 0, many.ctypes.data_as(ctypes.c_void_p), 64,
                                ctypes.byref(total)) == EINVAL
    assert lib.cm_batch_prepare(0, 0, many.ctypes.data_as(ctypes.c_void_p), 1,
                                ctypes.byref(total)) == OK
    many["m"][5] = 1 << 48  # a side of 2^48 elements
    assert lib.cm_batch_prepare(0, 0, many[5:].ctypes.data_as(ctypes.c_void_p), 1,
                                ctypes.byref(total)) == EINVAL


def test_timing_argument_errors():
    lib = cm.load()
    u = ctypes.c_uint32()
    d = ctypes.c_double()
    assert lib.cm_timing_start(0) == EINVAL
    assert lib.cm_timing_start((1 << 20) + 1) == EINVAL
    assert lib.cm_timing_stop(ctypes.byref(u), ctypes.byref(d), ctypes.byref(d), None, None,
                              None) == EINVAL


def test_server_argument_errors():
    lib = cm.load()
    P = ctypes.c_void_p
    h = ctypes.c_void_p()
    assert lib.cm_server_create(0, 1, None, 1 << 20, 8, 2, 64, ctypes.byref(h)) == EINVAL
    assert lib.cm_server_create(9, 1, P(0x1000), 1 << 20, 8, 2, 64, ctypes.byref(h)) == EDTYPE
    assert lib.cm_server_create(0, 1, P(0x1000), 255, 8, 2, 64, ctypes.byref(h)) == EINVAL
    assert lib.cm_server_create(0, 1, P(0x1000), 1 << 20, 0, 2, 64, ctypes.byref(h)) == EINVAL
    assert lib.cm_server_create(0, 1, P(0x1000), 1 << 20, 8, 17, 64, ctypes.byref(h)) == EINVAL
    assert lib.cm_server_create(0, 1, P(0x1000), 1 << 20, 8, 2, 65536, ctypes.byref(h)) == EINVAL
    assert lib.cm_server_create(0, 1, P(0x1000), 1 << 20, 8, 2, 64, None) == EINVAL
    assert h.value is None
    t = ctypes.c_uint64()
    n = ctypes.c_uint32()
    assert lib.cm_server_submit(None, P(0x1000), P(0x2000), 4, P(0x3000), P(0x4000), 4, None, 0,
                                ctypes.byref(t)) == EINVAL
    assert lib.cm_server_submit_host(None, P(0x1000), P(0x2000), 4, P(0x3000), P(0x4000), 4,
                                     P(0x5000), P(0x6000), ctypes.byref(t)) == EINVAL
    assert lib.cm_server_poll(None, None, 0, ctypes.byref(n), 0) == EINVAL
    assert lib.cm_server_release(None, 1) == EINVAL
    assert lib.cm_server_get_stats(None, None) == EINVAL
    assert lib.cm_server_destroy(None) == EINVAL
    assert cm.status_string(-9) == "every request slot is taken"
    assert cm.status_string(-10) == "canceled at shutdown"


def test_one_hip_runtime_whatever_the_import_order(tmp_path):
    """Loading the library before torch must not leave two HIP runtimes in
    the process (torch's streams and memory would be foreign to the
    library's launches).  Checked in a fresh interpreter from its mappings."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1303_4312_amd as cm\n"
        "cm.load()\n"
        "import torch\n"
        "paths = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
        "print(len(paths))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300, check=True).stdout.split()
    assert out[-1] == "1", f"HIP runtimes mapped: {out[-1]}"


def test_partition_ablation_argument_errors():
    lib = cm.load()
    P = ctypes.c_void_p
    ws = lib.cm_partition_ablation_workspace_size(64)
    assert ws >= 65 * 8 and ws % 256 == 0
    assert lib.cm_partition_ablation_workspace_size(1) == 0
    args = dict(A=P(0x1000), Av=None, m=100, B=P(0x2000), Bv=None, n=100, C=P(0x10000), Cv=None)

    def call(P_, part, bounds=P(0x20000), wsb=ws, kt=0):
        return lib.cm_merge_partition_ablation(kt, args["A"], None, 100, args["B"], None, 100,
                                               args["C"], None, P_, part, bounds, P(0x30000), wsb,
                                               None)
    assert call(63, 0) == EINVAL      # odd P
    assert call(0, 0) == EINVAL
    assert call(64, 2) == EINVAL      # unknown partition
    assert call(64, 0, bounds=None) == EINVAL
    assert call(64, 0, wsb=ws - 1) == ENOSPC
    assert call(64, 0, kt=9) == EDTYPE


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_host_co_rank_descending(dtype):
    rng = np.random.default_rng(8)
    for m, n in ((0, 0), (3, 0), (0, 4), (57, 91), (1000, 10)):
        A = np.sort(rng.integers(0, 12, m).astype(dtype))[::-1].copy()
        B = np.sort(rng.integers(0, 12, n).astype(dtype))[::-1].copy()
        for i in range(0, m + n + 1, max(1, (m + n) // 13)):
            assert cm.co_rank_host(i, A, B, descending=True) == \
                oracle.co_rank_brute(i, A, B, descending=True)


def test_descending_key_types_accepted():
    lib = cm.load()
    for kt in range(6):
        assert lib.cm_merge_workspace_size(kt, 1, 1000, 1000) > 0
        assert lib.cm_sort_workspace_size(kt, 1, 1000) > 0
    assert lib.cm_merge_workspace_size(6, 1, 1000, 1000) == 0
    # every key type has its own default tile configuration
    try:
        for kt in range(6):
            assert lib.cm_set_config(kt, 1, kt + 1) == 0
        for kt in range(6):
            assert lib.cm_get_config(kt, 1) == kt + 1
        assert lib.cm_set_config(6, 1, 0) == EDTYPE
    finally:
        for kt in range(6):
            lib.cm_set_config(kt, 1, -1)


def test_records_argument_errors():
    lib = cm.load()
    P = ctypes.c_void_p
    assert lib.cm_origin_codes(5, 0, None, None, None) == EINVAL
    assert lib.cm_origin_codes(1 << 31, 0, P(0x1000), None, None) == EINVAL
    assert lib.cm_origin_codes(0, 0, None, None, None) == OK
    assert lib.cm_origin_codes(100, 100, P(0x1000), P(0x1100), None) == EALIAS
    assert lib.cm_gather_records(P(0x1000), 10, P(0x2000), 5, P(0x3000), 5, 0, P(0x4000),
                                 None) == EINVAL
    assert lib.cm_gather_records(P(0x1000), 10, None, 5, P(0x3000), 5, 8, P(0x4000),
                                 None) == EINVAL
    assert lib.cm_gather_records(P(0x1000), 10, P(0x2000), 5, P(0x3000), 5, 8, P(0x2000),
                                 None) == EALIAS
    assert lib.cm_gather_records(None, 0, None, 0, None, 0, 8, None, None) == OK
    # records past 2^64 bytes: one output, but a side whose records overflow
    assert lib.cm_gather_records(P(0x1000), 1, P(0x2000), 5, P(0x3000), 5, 1 << 62,
                                 P(0x4000), None) == EINVAL


def test_copy_tiles_argument_errors():
    lib = cm.load()
    P = ctypes.c_void_p
    A, Av, B, Bv, C, Cv = (P(0x100000 * k) for k in range(1, 7))
    assert lib.cm_copy_tiles(-1, A, Av, 16, B, Bv, 16, C, Cv, None) == EINVAL
    assert lib.cm_copy_tiles(cm.config_count(), A, Av, 16, B, Bv, 16, C, Cv, None) == EINVAL
    assert lib.cm_copy_tiles(0, A, Av, 18, B, Bv, 16, C, Cv, None) == EINVAL  # m % 4
    assert lib.cm_copy_tiles(0, A, Av, 16, B, Bv, 14, C, Cv, None) == EINVAL  # n % 4
    assert lib.cm_copy_tiles(0, P(0x100004), Av, 16, B, Bv, 16, C, Cv, None) == EINVAL
    assert lib.cm_copy_tiles(0, None, Av, 16, B, Bv, 16, C, Cv, None) == EINVAL
    assert lib.cm_copy_tiles(0, A, Av, 1 << 33, B, Bv, 1 << 33, C, Cv, None) == EINVAL
    assert lib.cm_copy_tiles(0, A, Av, 16, B, Bv, 16, A, Cv, None) == EALIAS
    assert lib.cm_copy_tiles(0, A, Av, 16, B, Bv, 16, C, C, None) == EALIAS
    assert lib.cm_copy_tiles(0, None, None, 0, None, None, 0, None, None, None) == OK


def test_sort_default_tile_until_a_config_is_set():
    """Until cm_set_config is called for their (key type, payload): sorts
    of 4-byte keys use the 256 x 9 tile with payloads and 256 x 11 without,
    uint64 sorts 256 x 9, keys-only single merges 256 x 9, segmented
    batches 256 x 15; merges with payloads use tile 0.  Checked in a fresh
    interpreter (other tests here set configurations)."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1303_4312_amd as cm\n"
        "N = 1 << 28\n"
        "print(cm.tuning_get(cm.OP_SORT, 'uint32', True, N)[0],\n"
        "      cm.tuning_get(cm.OP_SORT, 'float32', False, N)[0],\n"
        "      cm.tuning_get(cm.OP_SORT, 'uint64', True, N)[0],\n"
        "      cm.tuning_get(cm.OP_MERGE, 'uint32', True, N)[0])\n"
        "cm.set_config('uint32', True, 0)\n"
        "print(cm.tuning_get(cm.OP_SORT, 'uint32', True, N)[0],\n"
        "      cm.tuning_get(cm.OP_SORT, 'uint32', False, N)[0])\n"
        "print(cm.tuning_get(cm.OP_MERGE, 'uint64', False, N)[0],\n"
        "      cm.tuning_get(cm.OP_SEGMENTED, 'uint32', False, N)[0])\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300, check=True).stdout.split("\n")
    assert out[0].split() == ["6", "1", "6", "0"]
    assert out[1].split() == ["0", "1"]
    assert out[2].split() == ["6", "2"]
    assert cm.config_info(6) == (256, 9)


def test_c_client_builds_against_the_header(tmp_path):
    """A C program (tests/c_abi_client.c) compiles against include/ and
    links against the shared library alone (run on the GPU by
    tests/test_c_client_gpu.py)."""
    from tests import c_client
    exe = c_client.build(str(tmp_path))
    assert os.path.exists(exe)


def test_server_struct_mirrors():
    """The binding's ctypes mirrors of cm_server_done / cm_server_stats have
    the sizes the library asserts (80 bytes each)."""
    from paper_1303_4312_amd import serve
    assert ctypes.sizeof(serve.ServerDone) == 80
    assert ctypes.sizeof(serve.ServerStats) == 80


def test_noalloc_refuses_merges_beyond_its_scratch():
    """The allocation-free merge checks its size against the scratch array
    before touching the device: too large is CM_ENOSPC, a bad key type
    CM_EDTYPE, lengths past 2^48 CM_EINVAL."""
    lib = cm.load()
    P = ctypes.c_void_p
    fake = P(1 << 44)
    assert lib.cm_stable_merge_pairs_noalloc(0, fake, fake, 1 << 40, fake, fake, 0, fake, fake, None) == ENOSPC
    assert lib.cm_stable_merge_pairs_noalloc(9, fake, fake, 10, fake, fake, 0, fake, fake, None) == EDTYPE
    assert lib.cm_stable_merge_pairs_noalloc(0, fake, fake, 1 << 48, fake, fake, 0, fake, fake, None) == EINVAL
    assert cm.NOALLOC_SCRATCH_BYTES == 4 << 20


@pytest.mark.usefixtures("restore_settings")
def test_sort_run_length():
    """The LDS run sort takes 4, 2 or 1 pass blocks per run, as many as keep
    two workgroups' runs (keys and payloads) within a CU's LDS."""
    lib = cm.load()
    for kt in range(6):
        assert lib.cm_set_config(kt, 0, -1) == 0 and lib.cm_set_config(kt, 1, -1) == 0
    assert cm.sort_run_length("uint32", True, 1 << 28) == 4 * 256 * 9     # 73,728 B per run
    assert cm.sort_run_length("float32", True, 1 << 20) == 4 * 256 * 9
    assert cm.sort_run_length("uint32", False, 1 << 28) == 4 * 256 * 11   # keys alone: 256 x 11
    assert cm.sort_run_length("uint64", True, 1 << 28) == 2 * 256 * 9     # 12 B per element
    cm.tuning_set(cm.OP_SORT, "uint32", True, 29, 2, 0, 2)  # 256 x 15
    try:
        assert cm.sort_run_length("uint32", True, 1 << 28) == 2 * 256 * 15
    finally:
        cm.tuning_clear()
    assert lib.cm_sort_run_length(6, 1, 1000) == 0
