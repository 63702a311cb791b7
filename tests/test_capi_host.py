"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/jevd.h declares, and its host logic (argument
validation, orderings, defaults, messages) is right."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1008_0201_amd import jevd as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "jevd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert {"jacobi_evd", "jevd_create", "jevd_destroy", "jevd_strerror"} <= names
    L = B.lib()
    for name in names:
        assert hasattr(L, name), name
    assert names == set(B.EXPORTS)


def test_strerror_and_defaults():
    assert B.jevd_strerror(0) == "success"
    assert "max_sweeps" in B.jevd_strerror(-3)
    assert B.jevd_strerror(12345) == "unknown status"
    o = B.jevd_default_opts()
    assert (o.ordering, o.variant, o.block, o.max_sweeps, o.max_inner, o.accumulate_v) == (2, 3, 0, 50, 30, 0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 17, 64, 255, 256, 1024])
@pytest.mark.parametrize("kind", [1, 2])
def test_library_ordering_matches_oracle(orc, n, kind):
    lib_steps = B.jevd_ordering(n, kind)
    orc_steps = orc.ordering(n, kind)
    assert len(lib_steps) == len(orc_steps)
    for a, b in zip(lib_steps, orc_steps):
        assert sorted(a) == sorted(b)
        assert all(i < j for i, j in a)


@pytest.mark.parametrize("args,ok", [
    (dict(m=10, n=8, ldg=10), True),
    (dict(m=7, n=8, ldg=10), False),           # m < n
    (dict(m=10, n=0, ldg=10), False),          # n < 1
    (dict(m=10, n=8, ldg=9), False),           # ldg < m
    (dict(m=10, n=8, ldg=10, J=[1, -1] * 4), True),
    (dict(m=10, n=8, ldg=10, J=[1, 0] * 4), False),   # J entry not +-1
    (dict(m=10, n=8, ldg=10, J=[1, 2] * 4), False),
    (dict(m=10, n=8, ldg=10, tol=float("nan")), False),
    (dict(m=10, n=8, ldg=10, tol=float("inf")), False),
    (dict(m=10, n=8, ldg=10, has_U=True, ldu=9), False),
    (dict(m=10, n=8, ldg=10, has_V=True, ldv=7), False),
    (dict(m=10, n=8, ldg=10, has_V=True, ldv=8), True),
    (dict(m=10, n=8, ldg=10, ordering=3), False),
    (dict(m=10, n=8, ldg=10, variant=4), False),
    (dict(m=10, n=8, ldg=10, max_sweeps=0), False),
    (dict(m=10, n=8, ldg=10, accumulate_v=1), False),          # resume needs V
    (dict(m=10, n=8, ldg=10, accumulate_v=1, has_V=True, ldv=8), True),
    (dict(m=10, n=8, ldg=10, block=24), False),                # unsupported width
])
def test_validate(args, ok):
    o = B.jevd_default_opts()
    for k in ("ordering", "variant", "block", "max_sweeps", "accumulate_v"):
        if k in args:
            setattr(o, k, args[k])
    J = args.get("J")
    Jb = None if J is None else np.array(J, dtype=np.int8).tobytes()
    st = B.jevd_validate(args["m"], args["n"], args["ldg"], Jb, args.get("tol", 0.0), o,
                         args.get("has_U", False), args.get("ldu", args["m"]),
                         args.get("has_V", False), args.get("ldv", args["n"]))
    assert (st == 0) == ok
    if not ok:
        assert st == B.JEVD_EINVAL


@pytest.mark.parametrize("n", [4, 16, 64, 200, 1024])
def test_ring_table_keeps_one_column_per_slot(n):
    """Modified modulus on even n runs the ring of Alg. 3.1: every workgroup
    slot (a fixed ring process) keeps exactly one of its two columns from one
    step to the next, and the processes end the sweep on the antidiagonal in
    reverse order (the pair sets themselves are checked against the oracle
    above)."""
    steps = B.jevd_ordering(n, B.ORD_MODMODULUS)
    p = n // 2
    for k in range(n - 1):
        for b in range(p):
            shared = set(steps[k][b]) & set(steps[k + 1][b])
            assert len(shared) == 1, (k, b, steps[k][b], steps[k + 1][b])
    first = {tuple(sorted(pr)) for pr in steps[0]}
    assert first == {(r, n - 1 - r) for r in range(p)}


def test_batch_entry_points_reject_null_arguments():
    """The batched entry points check their handles and arrays on the host
    before any device work (no GPU needed for these paths)."""
    L = B.lib()
    plan = ctypes.c_void_p(123)
    m = (ctypes.c_int * 1)(4)
    st = L.jevd_batch_create(None, 1, m, m, None, m, None, None, None, None, None, None, None,
                             None, ctypes.byref(plan))
    assert st == B.JEVD_EINVAL and plan.value is None
    assert L.jevd_batch_create(None, 1, m, m, None, m, None, None, None, None, None, None, None,
                               None, None) == B.JEVD_EINVAL
    assert L.jevd_batch_run(None, None) == B.JEVD_EINVAL
    assert L.jevd_batch_results(None, None, None) == B.JEVD_EINVAL
    assert L.jevd_batch_destroy(None) == B.JEVD_OK
    assert L.jacobi_evd_batched(None, 1, m, m, None, m, None, None, None, None, None, None, None,
                                None, None, None) == B.JEVD_EINVAL


def test_adjoint_entry_points_reject_bad_arguments():
    """jevd_canonicalize and jevd_adjoint check sizes and pointers on the
    host before any device work."""
    L = B.lib()
    vp = ctypes.c_void_p
    # null handle
    assert L.jevd_canonicalize(None, 1, 4, 4, vp(8), 4, vp(8), 4, 16, None, 4, 16, vp(8), vp(8),
                               None) == B.JEVD_EINVAL
    assert L.jevd_adjoint(None, 1, 4, 4, vp(8), 4, 16, None, 4, vp(8), 4, vp(8), 4, 16, None, 4,
                          None, 4, 16, vp(8), 4, 16) == B.JEVD_EINVAL
    assert B.jevd_strerror(B.JEVD_EINVAL)


def test_opts_struct_matches_header():
    """The binding's jevd_opts / jevd_info layouts follow include/jevd.h."""
    import re
    hdr = open(os.path.join(ROOT, "include", "jevd.h")).read()
    opts = hdr[hdr.index("typedef struct {"):hdr.index("} jevd_opts;")]
    fields = re.findall(r"^\s+int (\w+);", opts, re.M)
    assert fields == [f for f, _ in B.jevd_opts._fields_]
    start = hdr.index("typedef struct {", hdr.index("JEVD_INFO_MAX_SWEEPS"))
    info = hdr[start:hdr.index("} jevd_info;")]
    info = re.sub(r"/\*.*?\*/", "", info, flags=re.S)
    names = re.findall(r"^\s+(?:int|long long|double) (\w+)(?:\[\w+\])?;", info, re.M)
    assert names == [f for f, _ in B.jevd_info._fields_]
    o = B.jevd_default_opts()
    assert (o.ordering, o.variant, o.block, o.max_sweeps, o.max_inner, o.accumulate_v, o.pivot,
            o.precision) == (B.ORD_MODMODULUS, B.VAR_AUTO, 0, 50, 30, 0, B.PIVOT_NONE, B.PREC_FP64)
    for bad in (dict(pivot=2), dict(precision=2), dict(pivot=1, variant=0), dict(precision=1, variant=0)):
        o = B.jevd_default_opts()
        for k, v in bad.items():
            setattr(o, k, v)
        assert B.jevd_validate(64, 64, 64, None, 0.0, o, False, 64, False, 64) == B.JEVD_EINVAL, bad
    o = B.jevd_default_opts()
    o.variant, o.block, o.precision = 1, 16, 1
    J = bytes([1] * 63 + [255])
    assert B.jevd_validate(64, 64, 64, J, 0.0, o, False, 64, False, 64) == B.JEVD_EINVAL
    assert B.jevd_validate(64, 64, 64, None, 0.0, o, False, 64, False, 64) == B.JEVD_OK


@pytest.mark.parametrize("m,n,variant,block,pivot,ok", [
    (256, 256, 1, 16, 0, True), (256, 256, 1, 32, 0, True), (256, 256, 1, 64, 0, True),
    (256, 256, 2, 64, 0, True),
    (256, 256, 1, 64, 1, False),        # b = 64 runs the unpivoted pivot solve only
    (256, 256, 2, 32, 1, True),         # sign pivoting at b <= 32
    (1000, 1000, 1, 32, 0, True),       # uneven partition: 32 blocks of 31 or 32 columns
    (1030, 1030, 2, 64, 0, True),       # 18 blocks of 57 or 58 columns
    (1000, 1000, 1, 32, 1, False),      # sign pivoting needs n divisible by 2b
    (70, 70, 1, 32, 0, True),           # 4 blocks of 17 or 18 columns (each <= b)
    (3, 3, 1, 16, 0, True), (2, 2, 2, 16, 0, True),
    (1, 1, 1, 16, 0, False),            # a block pivot needs two columns
    (1000, 1000, 1, 24, 0, False), (1000, 1000, 1, 128, 0, False),   # unsupported widths
])
def test_block_options_as_documented(m, n, variant, block, pivot, ok):
    """Each value the header documents for opts.block / opts.pivot with the
    block variants is accepted or rejected as documented (Sec. 3: widths of
    the uniform partition differ by at most one)."""
    o = B.jevd_default_opts()
    o.variant, o.block, o.pivot = variant, block, pivot
    st = B.jevd_validate(m, n, m, None, 0.0, o, False, m, False, n)
    assert (st == B.JEVD_OK) == ok, st


def test_tune_table_record_lookup_and_file(tmp_path):
    """The autotuner's table: records persist in the tune file, the last
    record of a shape wins, invalid records are refused, and block = 0
    follows the record (here: b = 64 for 256 x 256, which then refuses sign
    pivoting)."""
    path = str(tmp_path / "tune.txt")
    assert B.jevd_tune_file(path) == B.JEVD_OK
    try:
        assert B.jevd_tune_lookup(256, 256)[0] == B.JEVD_EINVAL
        assert B.jevd_tune_record(256, 256, 32, B.VAR_FULL_BLOCK, 12.5) == B.JEVD_OK
        assert B.jevd_tune_record(256, 256, 64, B.VAR_BLOCK_ORIENTED, 10.0) == B.JEVD_OK
        assert B.jevd_tune_record(1024, 1024, 0, B.VAR_POINTWISE, 60.0) == B.JEVD_OK
        assert B.jevd_tune_record(256, 256, 24, B.VAR_BLOCK_ORIENTED, 1.0) == B.JEVD_EINVAL
        assert B.jevd_tune_record(256, 256, 32, B.VAR_POINTWISE, 1.0) == B.JEVD_EINVAL
        assert B.jevd_tune_record(256, 256, 32, B.VAR_AUTO, 1.0) == B.JEVD_EINVAL
        assert B.jevd_tune_record(256, 256, 32, B.VAR_BLOCK_ORIENTED, -1.0) == B.JEVD_EINVAL
        assert B.jevd_tune_lookup(256, 256) == (B.JEVD_OK, 64, B.VAR_BLOCK_ORIENTED, 10.0)
        lines = open(path).read().split("\n")
        assert "256 256 64 1 10.000000" in lines and "1024 1024 0 0 60.000000" in lines
        # a fresh load of the file gives the same table
        assert B.jevd_tune_file(path) == B.JEVD_OK
        assert B.jevd_tune_lookup(256, 256) == (B.JEVD_OK, 64, B.VAR_BLOCK_ORIENTED, 10.0)
        assert B.jevd_tune_lookup(1024, 1024) == (B.JEVD_OK, 0, B.VAR_POINTWISE, 60.0)
        o = B.jevd_default_opts()          # variant AUTO, block 0
        assert B.jevd_validate(256, 256, 256, None, 0.0, o, False, 256, False, 256) == B.JEVD_OK
        # block 0 takes the recorded b = 64, which has no sign pivoting
        o.variant, o.pivot = B.VAR_BLOCK_ORIENTED, B.PIVOT_SIGN
        assert B.jevd_validate(256, 256, 256, None, 0.0, o, False, 256, False, 256) == B.JEVD_EINVAL
        o.block = 32
        assert B.jevd_validate(256, 256, 256, None, 0.0, o, False, 256, False, 256) == B.JEVD_OK
        # an unreadable line is skipped, the rest is kept
        with open(path, "a") as f:
            f.write("garbage line\n512 512 32 2 3.5\n")
        assert B.jevd_tune_file(path) == B.JEVD_OK
        assert B.jevd_tune_lookup(512, 512) == (B.JEVD_OK, 32, B.VAR_FULL_BLOCK, 3.5)
    finally:
        B.jevd_tune_file(str(tmp_path / "empty.txt"))


def test_auto_variant_untuned_shapes(tmp_path):
    """Without a record, JEVD_VAR_AUTO is pointwise below n = 2048 (any n
    then validates) and block-oriented from n = 2048 (the block partition
    rules apply: sign pivoting is refused for a width that does not divide
    n evenly)."""
    B.jevd_tune_file(str(tmp_path / "none.txt"))
    o = B.jevd_default_opts()
    assert B.jevd_validate(1999, 1999, 1999, None, 0.0, o, False, 1999, False, 1999) == B.JEVD_OK
    o.pivot = B.PIVOT_SIGN
    # pointwise has no Cholesky: sign pivoting needs an explicit block variant
    assert B.jevd_validate(2048, 2048, 2048, None, 0.0, o, False, 2048, False, 2048) == B.JEVD_EINVAL
    o.variant = B.VAR_BLOCK_ORIENTED
    assert B.jevd_validate(2050, 2050, 2050, None, 0.0, o, False, 2050, False, 2050) == B.JEVD_EINVAL
    o.pivot = B.PIVOT_NONE
    assert B.jevd_validate(2050, 2050, 2050, None, 0.0, o, False, 2050, False, 2050) == B.JEVD_OK


def test_mfma_rate_rejects_bad_arguments():
    """jevd_mfma_f64_rate checks its arguments before any device work."""
    L = B.lib()
    t = ctypes.c_double(-1.0)
    assert L.jevd_mfma_f64_rate(None, 4, 16, ctypes.byref(t)) == B.JEVD_EINVAL
    fake = ctypes.c_void_p(1)   # never dereferenced: the argument checks come first
    for wps, iters in ((0, 16), (3, 16), (8, 16), (4, 0)):
        assert L.jevd_mfma_f64_rate(fake, wps, iters, ctypes.byref(t)) == B.JEVD_EINVAL
    assert L.jevd_mfma_f64_rate(fake, 4, 16, None) == B.JEVD_EINVAL
    assert t.value == -1.0


def test_batch_tune_table_record_lookup_and_file(tmp_path):
    """The batched solve's per-class records: kept, looked up, written to
    the table file beside the block records and read back; invalid records
    refused."""
    path = str(tmp_path / "tune.txt")
    try:
        assert B.jevd_tune_file(path) == B.JEVD_OK
        assert B.jevd_batch_tune_lookup(0)[0] == B.JEVD_EINVAL
        assert B.jevd_batch_tune_record(0, 4, 1.5) == B.JEVD_OK
        assert B.jevd_batch_tune_record(2, 8, 7.25) == B.JEVD_OK
        assert B.jevd_batch_tune_record(2, 16, 6.0) == B.JEVD_OK      # the last record wins
        assert B.jevd_tune_record(512, 512, 32, 1, 3.0) == B.JEVD_OK  # a block record beside them
        for bad in ((-1, 4, 1.0), (B.BATCH_CLASSES, 4, 1.0), (1, 3, 1.0), (1, 32, 1.0),
                    (1, 8, -1.0)):
            assert B.jevd_batch_tune_record(*bad) == B.JEVD_EINVAL, bad
        text = open(path).read()
        assert "batch 0 4 " in text and "batch 2 16 " in text and "batch 2 8 " not in text
        assert B.jevd_tune_file(path) == B.JEVD_OK   # reload from the file
        assert B.jevd_batch_tune_lookup(0)[:2] == (B.JEVD_OK, 4)
        assert B.jevd_batch_tune_lookup(2)[:2] == (B.JEVD_OK, 16)
        assert B.jevd_batch_tune_lookup(1)[0] == B.JEVD_EINVAL
        assert B.jevd_tune_lookup(512, 512)[:3] == (B.JEVD_OK, 32, 1)
    finally:
        B.jevd_tune_file(None)


def test_batch_tuning_entry_points_reject_bad_arguments():
    L = B.lib()
    w = (ctypes.c_int * B.BATCH_CLASSES)()
    assert L.jevd_batch_waves(None, w) == B.JEVD_EINVAL
    assert L.jevd_batch_autotune(None, 1, w) == B.JEVD_EINVAL
    fake = ctypes.c_void_p(1)   # never dereferenced: the argument checks come first
    assert L.jevd_batch_autotune(fake, 2, w) == B.JEVD_EINVAL
