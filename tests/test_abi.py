"""CPU-side checks of the C ABI library: it loads, exports every function that
include/spx.h declares, rejects bad arguments before touching the GPU, and the
Python layer fails loudly when the library is missing."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "spx.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    from paper_1302_1078_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1302_1078_amd import build
        build.build()
    return _lib.load()


def test_header_lists_the_entry_points():
    names = header_functions()
    for must in ("csr_spmv", "csr_spmm", "csr_from_coo", "csr_plan_create", "csr_spmv_t", "csr_sddmm",
                 "csr_transpose_index", "csr_batch_create", "csr_batch_run", "spx_last_error"):
        assert must in names
    assert len(names) >= 22


def test_every_declared_symbol_is_exported(lib):
    from paper_1302_1078_amd import _lib
    for name in header_functions():
        assert getattr(lib, name, None) is not None, name
    assert set(header_functions()) == set(_lib.SIGNATURES)


def test_argument_errors_without_gpu(lib):
    from paper_1302_1078_amd import _lib
    o = _lib.PlanOpts()
    assert lib.spx_plan_default_opts(0, 0, ctypes.byref(o)) == _lib.SPX_ERR_INVALID
    assert b"k=0" in lib.spx_last_error()
    assert lib.spx_plan_default_opts(16, 0, ctypes.byref(o)) == _lib.SPX_OK and o.max_k == 16
    nb = ctypes.c_size_t()
    bad = _lib.PlanOpts.from_dict({"nbins": 3, "upper": [8, 4], "lanes": [1, 2, 4]})
    assert lib.csr_plan_workspace_bytes(10, 10, ctypes.byref(bad), ctypes.byref(nb)) == _lib.SPX_ERR_INVALID
    bad = _lib.PlanOpts.from_dict({"nbins": 2, "upper": [8], "lanes": [0, 4]})
    assert lib.csr_plan_workspace_bytes(10, 10, ctypes.byref(bad), ctypes.byref(nb)) == _lib.SPX_ERR_INVALID
    bad = _lib.PlanOpts.from_dict({"nbins": 1, "upper": [], "lanes": [128]})
    assert lib.csr_plan_workspace_bytes(10, 10, ctypes.byref(bad), ctypes.byref(nb)) == _lib.SPX_ERR_INVALID
    good = _lib.PlanOpts.from_dict({"nbins": 2, "upper": [8], "lanes": [4, 0], "split_chunk": 512})
    assert lib.csr_plan_workspace_bytes(1000, 9000, ctypes.byref(good), ctypes.byref(nb)) == _lib.SPX_OK
    assert nb.value >= 4 * 1000
    # sizes and dtype pairs are checked before any launch
    null = ctypes.c_void_p(0)
    assert lib.csr_spmv(-1, 4, 0, null, null, null, 0, null, null, 0, null, null) == _lib.SPX_ERR_INVALID
    assert lib.csr_spmv(4, 4, 0, null, null, null, 0, null, null, 1, null, null) == _lib.SPX_ERR_UNSUPPORTED
    assert lib.csr_spmv(0, 4, 0, null, null, null, 0, null, null, 0, null, null) == _lib.SPX_OK
    assert lib.csr_spmm(4, 4, 0, null, null, null, 0, 8, null, 4, null, 8, 0, null, null) == _lib.SPX_ERR_INVALID
    assert lib.csr_spmv_t(4, 4, 1, null, null, null, null, null, null, 0, 1, null, 1, null, 1, 0, 0, null,
                          null) == _lib.SPX_ERR_INVALID
    # leading dimensions below k are rejected for both modes, k = 1 included
    for mode in (0, 1):
        for lddy, lddx in ((0, 1), (1, 0)):
            assert lib.csr_spmv_t(4, 4, 0, null, null, null, null, null, null, 0, 1, null, lddy, null, lddx, 0,
                                  mode, null, null) == _lib.SPX_ERR_INVALID, (mode, lddy, lddx)
    for lddy, ldx in ((0, 1), (1, 0)):
        assert lib.csr_sddmm(4, 4, 0, null, null, 1, null, lddy, null, ldx, null, 0, null,
                             null) == _lib.SPX_ERR_INVALID, (lddy, ldx)
    assert lib.csr_from_coo_workspace_bytes(4, 4, -1, ctypes.byref(nb)) == _lib.SPX_ERR_INVALID
    assert lib.csr_from_coo(4, 4, 2, null, null, null, null, null, null, null, null, 0, null) == _lib.SPX_ERR_INVALID
    assert b"gfx950" in lib.spx_version()


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_1302_1078_amd._lib as L; L.LIB_PATH = '/nonexistent/libspx.so'; L._lib = None\n"
            "import paper_1302_1078_amd as P\n"
            "try:\n    P.version()\nexcept ImportError as e:\n    print('LOUD', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert "LOUD" in r.stdout, r.stderr


def test_occupancy_option_checked():
    """occupancy outside [0, 8] is rejected when the plan is sized (host-side check)."""
    import ctypes
    from paper_1302_1078_amd import _lib
    L = _lib.load()
    o = _lib.PlanOpts.from_dict({"nbins": 1, "upper": [], "lanes": [64], "max_k": 1, "occupancy": 9})
    nb = ctypes.c_size_t()
    assert L.csr_plan_workspace_bytes(100, 1000, ctypes.byref(o), ctypes.byref(nb)) != 0
    assert b"occupancy" in L.spx_last_error()
    o.occupancy = 4
    assert L.csr_plan_workspace_bytes(100, 1000, ctypes.byref(o), ctypes.byref(nb)) == 0
    o.row_period = -1
    assert L.csr_plan_workspace_bytes(100, 1000, ctypes.byref(o), ctypes.byref(nb)) != 0
    assert b"row_period" in L.spx_last_error()
    o.row_period = 0
    assert L.csr_plan_workspace_bytes(100000, 1000000, ctypes.byref(o), ctypes.byref(nb)) == 0
    plain = nb.value
    o.row_period = 1000   # eight band counts per bin and tile
    assert L.csr_plan_workspace_bytes(100000, 1000000, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value > plain


def test_plan_opts_roundtrip_and_autotune_cache(tmp_path):
    from paper_1302_1078_amd import _lib, autotune
    d = {"nbins": 3, "upper": [4, 64], "lanes": [4, 64, 0], "split_chunk": 1024, "kahan_len": 256,
         "max_k": 8, "flags": 0, "occupancy": 3, "row_period": 16384}
    assert _lib.PlanOpts.from_dict(d).to_dict() == d
    p = tmp_path / "c.json"
    p.write_text("{broken")
    assert autotune.load_cache(str(p)) == {}
    p.write_text("[1, 2]")
    assert autotune.load_cache(str(p)) == {}
    assert autotune._valid({"opts": {"nbins": 2, "upper": [3], "lanes": [1]}}) is None
    assert autotune._valid({"opts": d}) is not None
    assert autotune._valid({"nope": 1}) is None


def test_size_limits_checked_before_any_work(lib):
    """nnz above SPX_MAX_NNZ is refused as unsupported by every entry point
    that takes it, before any pointer is read (the kernels' int32 positions
    need the headroom); split_chunk above SPX_MAX_SPLIT_CHUNK is invalid."""
    from paper_1302_1078_amd import _lib
    big = 2**31 - 2**25 + 1
    null = ctypes.c_void_p(0)
    sz = ctypes.c_size_t()
    out = ctypes.c_void_p()
    o = _lib.PlanOpts.from_dict({"nbins": 2, "upper": [64], "lanes": [64, 0], "split_chunk": 4096, "max_k": 1})
    unsupported = 2
    calls = {
        "csr_spmv": lambda n: lib.csr_spmv(10, 10, n, null, null, null, 0, null, null, 0, null, null),
        "csr_spmm": lambda n: lib.csr_spmm(10, 10, n, null, null, null, 0, 4, null, 4, null, 4, 0, null, null),
        "csr_spmv_t": lambda n: lib.csr_spmv_t(10, 10, n, null, null, null, null, null, null, 0, 1, null, 1,
                                               null, 1, 0, 1, null, null),
        "csr_sddmm": lambda n: lib.csr_sddmm(10, 10, n, null, null, 1, null, 1, null, 1, null, 0, null, null),
        "csr_from_coo_workspace_bytes": lambda n: lib.csr_from_coo_workspace_bytes(10, 10, n, ctypes.byref(sz)),
        "csr_validate": lambda n: lib.csr_validate(10, 10, n, null, null, 0, null, null),
        "csr_transpose_index": lambda n: lib.csr_transpose_index(10, 10, n, null, null, null, null, null, null,
                                                                 0, null),
        "csr_plan_workspace_bytes": lambda n: lib.csr_plan_workspace_bytes(10, n, ctypes.byref(o), ctypes.byref(sz)),
        "csr_plan_create": lambda n: lib.csr_plan_create(10, 10, n, null, ctypes.byref(o), null, 0, null,
                                                         ctypes.byref(out)),
        "csr_degree_order": lambda n: lib.csr_degree_order(10, n, null, null, null, 0, null),
        "csr_csc_value_map": lambda n: lib.csr_csc_value_map(n, null, null, null, null, 0, null),
        "csr_values_to_csc": lambda n: lib.csr_values_to_csc(n, null, null, null, 0, null, null, null),
        "csr_permute": lambda n: lib.csr_permute(10, n, null, null, null, null, null, null, null, null, null, 0,
                                                 null),
    }
    for name, call in calls.items():
        assert call(big) == unsupported, name
        assert b"SPX_MAX_NNZ" in lib.spx_last_error(), name
    o.split_chunk = 2**24 + 1
    assert lib.csr_plan_workspace_bytes(10, 100, ctypes.byref(o), ctypes.byref(sz)) == 1
    assert b"split_chunk" in lib.spx_last_error()
    o.split_chunk = 2**24
    assert lib.csr_plan_workspace_bytes(10, 100, ctypes.byref(o), ctypes.byref(sz)) == 0


# ---------------------------------------------------------------- host assembly and validation

def test_from_coo_host_bit_exact_against_oracle(lib):
    """csr_from_coo_host (the library's host assembly, a two-pass counting
    sort) gives the oracle's CSR bit for bit: duplicates summed in input
    order, empty rows, shuffled input, m != n."""
    import numpy as np
    import oracle
    import paper_1302_1078_amd as spx
    import spgen
    rng = np.random.default_rng(3)
    cases = []
    base = spgen.powerlaw(3000, 2500, 2.0, 800, 12.0, seed=2)
    dup = rng.choice(base.r.size, base.r.size // 10, replace=False)
    r = np.concatenate([base.r, base.r[dup]])
    c = np.concatenate([base.c, base.c[dup]])
    v = np.concatenate([base.v, rng.uniform(-1, 1, dup.size)])
    p = rng.permutation(r.size)
    cases.append((base.m, base.n, r[p], c[p], v[p]))
    # 1e16 + 1 - 1e16: only the input order gives 0
    cases.append((2, 4, np.array([1, 1, 1, 0]), np.array([3, 3, 3, 0]), np.array([1e16, 1.0, -1e16, 2.0])))
    cases.append((5, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)))
    cases.append((0, 5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)))
    for m, n, r, c, v in cases:
        A = oracle.csr_from_coo(m, n, r, c, v)
        rowptr, colind, values = spx.from_coo_host(m, n, r, c, v)
        assert np.array_equal(rowptr, A.rowptr) and np.array_equal(colind, A.colind)
        assert np.array_equal(values.view(np.uint64), A.values.view(np.uint64))
        spx.validate_host(m, n, rowptr, colind)
    assert spx.from_coo_host(2, 4, *cases[1][2:])[2][1] == 0.0


def test_host_calls_reject_bad_input(lib):
    import numpy as np
    import paper_1302_1078_amd as spx
    from paper_1302_1078_amd._lib import SPX_ERR_INVALID, SpxError
    with pytest.raises(SpxError) as e:
        spx.from_coo_host(3, 3, [0, 3], [0, 1], [1.0, 2.0])
    assert e.value.status == SPX_ERR_INVALID and b"outside" in lib.spx_last_error()
    good = (np.array([0, 2, 2, 3]), np.array([0, 2, 1]))
    spx.validate_host(3, 3, *good)
    bad = [(np.array([1, 2, 2, 3]), good[1], b"rowptr[0]"),
           (np.array([0, 2, 2, 4]), good[1], b"rowptr[m]"),
           (np.array([0, 2, 1, 3]), good[1], b"row 1"),
           (good[0], np.array([0, 3, 1]), b"colind[1]"),
           (good[0], np.array([0, -1, 1]), b"colind[1]")]
    for rp, ci, what in bad:
        with pytest.raises(SpxError):
            spx.validate_host(3, 3, rp, ci)
        assert what in lib.spx_last_error(), what
    # rowptr[m] = nnz counts against the colind length the caller passes
    with pytest.raises(SpxError):
        spx.validate_host(3, 3, good[0], good[1][:2])


# The boundary's calls against the scope table's list: each listed call is
# exported under its listed name, or replaced by the named call(s) (reasons in
# the design notes): a device assembly and validation beside the host ones,
# and the per-matrix tuning record carried inside the batch descriptor.
BOUNDARY_MAP = {
    "csr_spmv": ["csr_spmv"],
    "csr_spmm": ["csr_spmm"],
    "csr_from_coo_host": ["csr_from_coo_host", "csr_from_coo"],
    "csr_validate_host": ["csr_validate_host", "csr_validate"],
    "csr_plan_workspace_bytes": ["csr_plan_workspace_bytes"],
    "csr_plan_create": ["csr_plan_create"],
    "csr_plan_export_bins": ["csr_plan_export_bins"],
    "csr_plan_destroy": ["csr_plan_destroy"],
    "csr_transpose_index": ["csr_transpose_index"],
    "csr_spmv_t": ["csr_spmv_t"],
    "csr_sddmm": ["csr_sddmm"],
    "csr_batch_create": ["csr_batch_create"],
    "csr_batch_run": ["csr_batch_run"],
    "csr_batch_destroy": ["csr_batch_destroy"],
    "spx_last_error": ["spx_last_error"],
}


def test_boundary_covers_the_scope_table(lib):
    names = set(header_functions())
    for listed, built in BOUNDARY_MAP.items():
        for b in built:
            assert b in names and getattr(lib, b, None) is not None, (listed, b)
    # spx_tune (variant + thresholds per matrix) is the spx_plan_opts carried
    # in each spx_csr_desc: csr_batch_create takes no separate host_tunes array
    from paper_1302_1078_amd import _lib
    fields = dict(_lib.CsrDesc._fields_)
    assert fields["opts"] is _lib.PlanOpts
    assert {"nbins", "upper", "lanes", "split_chunk", "kahan_len"} <= {f for f, _ in _lib.PlanOpts._fields_}
