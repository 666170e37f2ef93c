"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
validates arguments before any device work, and holds the paper's tables."""

import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "logm.h")

lm = pytest.importorskip("paper_2401_10089_amd")


@pytest.fixture(scope="module")
def lib():
    try:
        return lm.load_library()
    except lm.LibraryNotBuilt as e:
        pytest.fail(f"library not built: {e}")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(logm_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(lm.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_strerror(lib):
    assert "gfx950" in lm.version()
    for code, name in lm.STATUS.items():
        assert lm.strerror(code)
    assert lm.strerror(99) == "unknown status"


def test_default_opts(lib):
    o = lm.default_opts()
    assert (o.k_max, o.max_sqrt, o.db_max_iter, o.theta_source) == (9, 50, 30, 0)


def test_workspace_size(lib):
    sizes = [lm.workspace_size(n) for n in (1, 64, 65, 1000, 4096)]
    assert all(s > 0 for s in sizes)
    assert sizes == sorted(sizes)
    # eleven padded matrices dominate
    assert sizes[-1] >= 11 * 4096 * 4096 * 8
    b = ctypes.c_size_t(0)
    assert lib.logm_workspace_size(0, 0, None, ctypes.byref(b)) == 1
    assert lib.logm_workspace_size(7, 10, None, ctypes.byref(b)) == 1


FAKE = ctypes.c_void_p(0x10000)   # never dereferenced: validation fails first


def fwd(lib, dtype=0, n=8, A=FAKE, lda=8, L=FAKE, ldl=8, opts=None, ws=None, ws_bytes=0):
    return lib.logm_forward(dtype, n, A, lda, L, ldl, ctypes.byref(opts) if opts else None, None,
                            ws, ws_bytes, None)


def test_forward_argument_validation(lib):
    assert fwd(lib, n=0) == 1
    assert fwd(lib, A=None) == 1
    assert fwd(lib, L=None) == 1
    assert fwd(lib, lda=7) == 1
    assert fwd(lib, ldl=3) == 1
    assert fwd(lib, dtype=5) == 1
    assert fwd(lib, dtype=1, ws=FAKE, ws_bytes=100) == 3   # complex: workspace of the 2n run
    b_r, b_c = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.logm_workspace_size(0, 100, None, ctypes.byref(b_r)) == 0
    assert lib.logm_workspace_size(1, 100, None, ctypes.byref(b_c)) == 0
    assert b_c.value > 2 * b_r.value
    o = lm.default_opts()
    o.k_max = 10                                       # Table 2 ends at k = 9
    assert fwd(lib, opts=o) == 1
    o = lm.default_opts()
    o.max_sqrt = 65
    assert fwd(lib, opts=o) == 1
    o = lm.default_opts()
    o.reserved = 1
    assert fwd(lib, opts=o) == 1
    o = lm.default_opts()
    o.pivot_search = 2                                 # 0 or 1 only
    assert fwd(lib, opts=o) == 1
    o = lm.default_opts()
    o.graph_fp32 = 2                                   # 0 or 1 only
    assert fwd(lib, opts=o) == 1
    o = lm.default_opts()
    o.balance = 2                                      # 0 or 1 only
    assert fwd(lib, opts=o) == 1
    assert fwd(lib, ws=FAKE, ws_bytes=100) == 3        # workspace too small


def test_noalloc_argument_validation(lib):
    """The allocation-free entry point refuses bad sizes and pointers before any
    device work (n above its fixed scratch's 256 included)."""
    f = lib.logm_forward_noalloc
    assert f(0, FAKE, 1, FAKE, 1, None, None, None) == 1
    assert f(257, FAKE, 257, FAKE, 257, None, None, None) == 1
    assert f(4, None, 4, FAKE, 4, None, None, None) == 1
    assert f(4, FAKE, 4, None, 4, None, None, None) == 1
    assert f(4, FAKE, 3, FAKE, 4, None, None, None) == 1
    o = lm.default_opts()
    o.k_max = 0
    assert f(4, FAKE, 4, FAKE, 4, ctypes.byref(o), None, None) == 1


def test_component_argument_validation(lib):
    best = (ctypes.c_int32 * 2)()
    assert lib.logm_autotune(0, None, 0, None, best, None) == 1
    assert lib.logm_autotune(64, None, 0, None, None, None) == 1
    assert lib.logm_autotune(64, FAKE, 100, None, best, None) == 3
    assert lib.logm_balance_f64(0, FAKE, 4, FAKE, 4, FAKE, None, None, None, 0, None) == 1
    assert lib.logm_balance_f64(4, FAKE, 4, FAKE, 3, FAKE, None, None, None, 0, None) == 1
    assert lib.logm_balance_f64(4, FAKE, 4, FAKE, 4, None, None, None, None, 0, None) == 1
    assert lib.logm_balance_f64(4, FAKE, 4, FAKE, 5, FAKE, None, None, None, 0, None) == 1   # in place needs lda == ldb
    assert lib.logm_gemm_f64(0, 4, 4, 1.0, FAKE, 4, FAKE, 4, 0.0, FAKE, 4, None) == 1
    assert lib.logm_gemm_f64(4, 4, 4, 1.0, FAKE, 3, FAKE, 4, 0.0, FAKE, 4, None) == 1
    assert lib.logm_inverse_f64(4, None, 4, FAKE, 4, None, None, 0, None) == 1
    assert lib.logm_sqrt_f64(4, FAKE, 4, FAKE, 4, 0, None, None, 0, None) == 1
    assert lib.logm_poly_f64(4, 10, 0, FAKE, 4, FAKE, 4, FAKE, 4, None, 0, None) == 1
    assert lib.logm_poly_f64(4, 5, -1, FAKE, 4, FAKE, 4, FAKE, 4, None, 0, None) == 1
    est = ctypes.c_double(0)
    assert lib.logm_normest_f64(4, FAKE, 4, FAKE, 4, 0, 0, ctypes.byref(est), None, None, 0, None) == 1
    assert lib.logm_normest_f64(4, FAKE, 4, FAKE, 4, 1, 2, ctypes.byref(est), None, None, 0, None) == 1


def test_backward_argument_validation(lib):
    b = ctypes.c_size_t(0)
    assert lib.logm_backward_workspace_size(0, 64, None, ctypes.byref(b)) == 0
    fwd_b = ctypes.c_size_t(0)
    assert lib.logm_workspace_size(0, 64, None, ctypes.byref(fwd_b)) == 0
    # forward workspace + (50 + 2 * 30 + 26) padded matrices
    assert b.value >= fwd_b.value + (50 + 60 + 26) * 64 * 64 * 8
    assert lib.logm_backward_workspace_size(0, 0, None, ctypes.byref(b)) == 1

    def call(dtype=0, n=8, A=FAKE, lda=8, G=FAKE, ldg=8, gA=FAKE, ldga=8, opts=None, ws=FAKE,
             ws_bytes=100):
        return lib.logm_backward(dtype, n, A, lda, G, ldg, gA, ldga,
                                 ctypes.byref(opts) if opts else None, None, ws, ws_bytes, None)

    assert call(n=0) == 1
    assert call(A=None) == 1
    assert call(G=None) == 1
    assert call(gA=None) == 1
    assert call(ldg=7) == 1
    assert call(ldga=7) == 1
    assert call(dtype=1) == 3                          # complex: workspace of the 2n run
    o = lm.default_opts()
    o.k_max = 10
    assert call(opts=o) == 1
    assert call() == 3                                 # workspace too small
    # taped pair: the workspace is required (it carries the tape)
    assert lib.logm_forward_taped(0, 8, FAKE, 8, FAKE, 8, None, None, None, 0, None) == 1
    assert lib.logm_forward_taped(0, 8, FAKE, 8, FAKE, 8, None, None, FAKE, 100, None) == 3
    assert lib.logm_backward_taped(0, 8, FAKE, 8, FAKE, 8, None, None, None, 0, None) == 1
    assert lib.logm_backward_taped(0, 8, FAKE, 7, FAKE, 8, None, None, FAKE, 100, None) == 1
    o = lm.default_opts()
    o.balance = 1
    assert lib.logm_forward_taped(0, 8, FAKE, 8, FAKE, 8, ctypes.byref(o), None, FAKE, 100, None) == 1


def test_batched_argument_validation(lib):
    b = ctypes.c_size_t(0)
    assert lib.logm_batched_workspace_size(3, 300, 10, ctypes.byref(b)) == 0
    assert b.value >= 13 * 300 * 8
    assert lib.logm_batched_workspace_size(0, 300, 10, ctypes.byref(b)) == 1
    assert lib.logm_batched_workspace_size(3, 300, 129, ctypes.byref(b)) == 1   # n <= 128
    assert lib.logm_batched_workspace_size(3, 0, 10, ctypes.byref(b)) == 1

    def call(batch=3, n_max=10, total=300, dims=FAKE, offs=FAKE, A=FAKE, L=FAKE, opts=None,
             st=FAKE, ws=FAKE, ws_bytes=1 << 20):
        return lib.logm_batched_f64(batch, n_max, total, dims, offs, A, L,
                                    ctypes.byref(opts) if opts else None, st, ws, ws_bytes, None)

    assert call(batch=0) == 1
    assert call(n_max=129) == 1
    assert call(dims=None) == 1
    assert call(offs=None) == 1
    assert call(A=None) == 1
    assert call(L=None) == 1
    assert call(st=None) == 1
    assert call(ws=None) == 1
    o = lm.default_opts()
    o.graph_fp32 = 1                                   # fp64 only on this path
    assert call(opts=o) == 1
    o = lm.default_opts()
    o.balance = 1                                      # no balancing on this path
    assert call(opts=o) == 1
    o = lm.default_opts()
    o.k_max = 10
    assert call(opts=o) == 1
    assert call(ws_bytes=100) == 3


def test_batched_autotune_argument_validation(lib):
    best = ctypes.c_int32(0)
    ms = ctypes.c_double(0)

    def call(**kw):
        a = dict(batch=4, n_max=100, total=1000, ws_bytes=1 << 40, best=ctypes.byref(best))
        a.update(kw)
        return lib.logm_batched_autotune(a["batch"], a["n_max"], a["total"], FAKE, FAKE, FAKE, FAKE, None,
                                         FAKE, FAKE, a["ws_bytes"], None, a["best"], ctypes.byref(ms))

    assert call(best=None) == 1
    assert call(n_max=129) == 1
    assert call(batch=0) == 1
    assert call(ws_bytes=100) == 3
    assert lib.logm_batched_set_split(0) == -1
    assert lib.logm_batched_set_split(65) == -1


def test_batched_c128_argument_validation(lib):
    by = ctypes.c_size_t(0)
    assert lib.logm_batched_c128_workspace_size(4, 100, 64, ctypes.byref(by)) == 0
    b_real = ctypes.c_size_t(0)
    assert lib.logm_batched_workspace_size(4, 400, 128, ctypes.byref(b_real)) == 0
    assert by.value >= b_real.value + 2 * 400 * 8          # the real run plus both representations
    assert lib.logm_batched_c128_workspace_size(4, 100, 65, ctypes.byref(by)) == 1   # 2n > 128
    assert lib.logm_batched_c128_workspace_size(0, 100, 8, ctypes.byref(by)) == 1
    assert lib.logm_batched_c128_workspace_size(4, 100, 8, None) == 1

    def call(**kw):
        a = dict(batch=4, n_max=8, total=100, dims=FAKE, offs=FAKE, A=FAKE, L=FAKE, opts=None,
                 status=FAKE, ws=FAKE, ws_bytes=1 << 40)
        a.update(kw)
        o = a["opts"]
        return lib.logm_batched_c128(a["batch"], a["n_max"], a["total"], a["dims"], a["offs"], a["A"],
                                     a["L"], ctypes.byref(o) if o is not None else None, a["status"],
                                     a["ws"], a["ws_bytes"], None)

    assert call(n_max=65) == 1
    assert call(dims=None) == 1
    assert call(A=None) == 1
    assert call(ws=None) == 1
    assert call(ws_bytes=100) == 3
    o = lm.default_opts()
    o.graph_fp32 = 1
    assert call(opts=o) == 1
    o = lm.default_opts()
    o.balance = 1
    assert call(opts=o) == 1


def test_library_table1_matches_paper(golden):
    t = golden("table1_k5.txt")
    h, g, y, m, th = lm.scheme(5)
    exp_h = [float(t[f"h_{j}_{i}"][0]) for j in range(2, 6) for i in range(2, j + 2)]
    exp_g = [float(t[f"g_{j}_{i}"][0]) for j in range(2, 6) for i in range(2, j + 2)]
    assert h == exp_h and g == exp_g
    assert y == [float(t[f"y_{q}"][0]) for q in range(1, 8)]
    assert (m, th) == (14, 0.246)


def test_library_table2_matches_paper(golden):
    t = golden("table2_theta.txt")
    for k in (1, 2, 3, 4, 5, 6, 7, 8, 9):
        m, _, theta = t[str(k)]
        _, _, _, mk, thk = lm.scheme(k)
        # k = 7, 8, 9: the fits' own Theta, below the printed values (reading R1)
        assert (mk, thk) == (int(m), oracle.THETA_DEFAULT[k][1])
        assert thk == (float(theta) if k <= 6 else oracle.THETA_FIT[k])
    assert lm.scheme(5, theta_source=1)[4] == 0.2448
    # Theta_6 recomputed for the library's own six-product fit (rounded down)
    assert lm.scheme(6, theta_source=1)[4] == oracle.THETA_FIT[6]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 7, 8, 9])
def test_library_taylor_schemes_expand_to_taylor(k):
    """The library's own k = 1, 2, 3, 4, 6..9 coefficients expand to T_{m_k} (exact
    rationals; k = 4 matches orders up to m_4 = 14 of its degree 16, k = 6..9 orders
    up to 20, 24, 27, 28 of their degrees 64..512)."""
    from fractions import Fraction

    from exact_poly import expand_rows

    h, g, y, m, _ = lm.scheme(k)
    rows_h, rows_g, pos = {}, {}, 0
    for j in range(2, k + 1):
        rows_h[j], rows_g[j] = h[pos:pos + j], g[pos:pos + j]
        pos += j
    z = expand_rows(k, rows_h, rows_g, y)
    for i in range(1, m + 1):
        assert abs(float((z[i] - Fraction(1, i)) * i)) <= (16 if k >= 4 else 4) * 2.0 ** -53


def test_library_k3_agrees_with_oracle():
    h, g, y, _, _ = lm.scheme(3)
    oh, og, oy = oracle.scheme_coefficients(3)
    flat_h = [v for j in (2, 3) for v in oh[j]]
    flat_g = [v for j in (2, 3) for v in og[j]]
    assert h == pytest.approx(flat_h, rel=1e-15, abs=1e-16)
    assert g == pytest.approx(flat_g, rel=1e-15, abs=1e-16)
    assert y == pytest.approx(list(oy), rel=1e-15, abs=1e-16)


def test_profile_calls_without_gpu(lib):
    lm.profile_enable(False)
    lm.profile_reset()
    p = lm.profile_get()
    assert p == {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0}


def test_product_path_has_no_oracle_import():
    """The binding and the package never reach the oracle (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2401_10089_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            src = open(os.path.join(pkg, name)).read()
            assert "import oracle" not in src and "from oracle" not in src, name
