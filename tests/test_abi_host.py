"""C-ABI tests that need no GPU: the library loads, exports every symbol
declared in include/wq.h, and its host-only calls validate inputs and
compute sizes and quadrature points (no compute calls)."""
import ctypes as C
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1605_01238_amd", "libwq.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libwq.so not built")


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "wq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wq_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    from paper_1605_01238_amd import _wq
    names = declared_symbols()
    assert len(names) >= 15
    lib = C.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == {s[0] for s in _wq.SIGNATURES}
    assert _wq.wq_version().startswith(b"wq-gfx950")


def make(knots3, p, prec=0, d=None):
    from paper_1605_01238_amd import _wq
    ks = [np.ascontiguousarray(k, dtype=np.float64) for k in knots3]
    n_knots = (C.c_int64 * len(ks))(*[len(k) for k in ks])
    ptrs = (C.POINTER(C.c_double) * len(ks))(*[k.ctypes.data_as(C.POINTER(C.c_double)) for k in ks])
    h = C.c_void_p()
    st = _wq.wq_plan_create(len(ks) if d is None else d, p, n_knots, ptrs, prec, C.byref(h))
    return st, h


@pytest.mark.parametrize("p,nel", [(2, (8, 9)), (4, (32, 17)), (6, (64, 64))])
def test_sizes_2d(p, nel):
    """A plane plan: the third direction is the trivial one (one function,
    one point), so the counts are those of the two real directions."""
    from paper_1605_01238_amd import _wq
    from workloads import Workload, open_uniform_knots
    st, h = make([open_uniform_knots(p, e) for e in nel], p)
    assert st == 0
    s = _wq.wq_sizes_t()
    assert _wq.wq_sizes(h, C.byref(s)) == 0
    w = Workload("t", p, nel, None, None)
    assert s.nnz == w.exact_nnz()
    assert tuple(s.n) == w.n_dof() + (1,)
    assert tuple(s.n_qp) == tuple(2 * e + 2 * p - 1 for e in nel) + (1,)
    assert s.n_rows == w.n_dof()[0] * w.n_dof()[1]
    x = np.zeros(64)
    assert _wq.wq_qpoints(h, 2, x.ctypes.data_as(C.POINTER(C.c_double))) == _wq.WQ_EINVAL
    _wq.wq_plan_destroy(h)
    good = open_uniform_knots(p, 8)
    assert make([good], p, d=0)[0] == _wq.WQ_EINVAL
    assert make([good] * 4, p, d=4)[0] == _wq.WQ_EINVAL


@pytest.mark.parametrize("p,nel", [(2, 5), (4, 33), (6, 1000)])
def test_sizes_1d(p, nel):
    """A curve plan: directions 2 and 3 are trivial; a row has #I_i1 entries
    (Section 3 count in one direction)."""
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    st, h = make([open_uniform_knots(p, nel)], p)
    assert st == 0
    s = _wq.wq_sizes_t()
    assert _wq.wq_sizes(h, C.byref(s)) == 0
    n = nel + p
    assert tuple(s.n) == (n, 1, 1) and s.n_rows == n
    assert tuple(s.n_qp) == (2 * nel + 2 * p - 1, 1, 1)
    assert s.nnz == (2 * p + 1) * n - p * (p + 1)
    assert s.nnz == sum(min(n - 1, i + p) - max(0, i - p) + 1 for i in range(n))
    _wq.wq_plan_destroy(h)


@pytest.mark.parametrize("p,nel", [(2, (8, 8, 8)), (4, (32, 32, 32)), (6, (64, 64, 64)), (3, (5, 7, 9))])
def test_sizes(p, nel):
    from paper_1605_01238_amd import _wq
    from workloads import Workload, open_uniform_knots
    st, h = make([open_uniform_knots(p, e) for e in nel], p)
    assert st == 0
    s = _wq.wq_sizes_t()
    assert _wq.wq_sizes(h, C.byref(s)) == 0
    w = Workload("t", p, nel, None, None)
    assert s.nnz == w.exact_nnz()
    assert tuple(s.n) == w.n_dof()
    assert tuple(s.n_qp) == tuple(2 * e + 2 * p - 1 for e in nel)
    assert s.value_bytes == 8 * s.nnz and s.workspace_bytes > 0
    _wq.wq_plan_destroy(h)


@pytest.mark.parametrize("p,nel,uniform", [(2, 8, True), (5, 9, False), (6, 11, True)])
def test_host_quadrature_points_match_oracle(p, nel, uniform):
    from oracle.rules import quadrature_points
    from oracle.splines import exact_knots
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots, random_open_knots
    k = open_uniform_knots(p, nel) if uniform else random_open_knots(p, nel, seed=7)
    st, h = make([k, k, k], p)
    assert st == 0
    x = np.zeros(2 * nel + 2 * p - 1)
    assert _wq.wq_qpoints(h, 1, x.ctypes.data_as(C.POINTER(C.c_double))) == 0
    ref = np.array([float(v) for v in quadrature_points(exact_knots(list(k)), p)])
    assert np.abs(x - ref).max() <= 4e-16
    _wq.wq_plan_destroy(h)


def test_invalid_inputs_rejected():
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    good = open_uniform_knots(3, 6)
    assert make([good] * 3, 1)[0] == _wq.WQ_EINVAL            # p below the minimum
    assert make([good] * 3, 7)[0] == _wq.WQ_EINVAL            # p above the maximum
    assert make([good] * 3, 3, prec=5)[0] == _wq.WQ_EINVAL    # precision
    bad = good.copy(); bad[5], bad[6] = bad[6], bad[5]        # decreasing
    assert make([good, bad, good], 3)[0] == _wq.WQ_EKNOTS
    notopen = good.copy(); notopen[0] = -0.1
    assert make([notopen, good, good], 3)[0] == _wq.WQ_EKNOTS
    rep = good.copy(); rep[5] = rep[6]                        # repeated interior knot (C^{p-2})
    assert make([good, good, rep], 3)[0] == _wq.WQ_EKNOTS
    few = open_uniform_knots(3, 4)                            # fewer than p+2 spans
    assert make([good, few, good], 3)[0] == _wq.WQ_EKNOTS
    nan = good.copy(); nan[4] = np.nan
    assert make([good, good, nan], 3)[0] == _wq.WQ_EKNOTS
    # the failed creation's message names the knot vector and the check
    assert make([good, good, rep], 3)[0] == _wq.WQ_EKNOTS
    msg = _wq.wq_last_error(None).decode()
    assert "knot vector 2" in msg and "simple" in msg, msg
    assert make([good, few, good], 3)[0] == _wq.WQ_EKNOTS
    assert "knot vector 1" in _wq.wq_last_error(None).decode()
    h = C.c_void_p()
    assert _wq.wq_plan_create(3, 3, None, None, 0, C.byref(h)) == _wq.WQ_EINVAL


def test_state_and_workspace_errors_without_device():
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    st, h = make([open_uniform_knots(2, 5)] * 3, 2)
    assert st == 0
    dummy = C.c_void_p(256)
    # assemble/setup/pattern before bind: state errors, no device call
    assert _wq.wq_assemble(h, _wq.WQ_STIFF, None, dummy, None) == _wq.WQ_ESTATE
    assert _wq.wq_setup(h, dummy, None, None) == _wq.WQ_ESTATE
    assert _wq.wq_pattern(h, dummy, dummy, None) == _wq.WQ_ESTATE
    assert _wq.wq_assemble(h, 4, None, None, None) == _wq.WQ_EINVAL
    assert _wq.wq_assemble(h, _wq.WQ_MASS, None, None, None) == _wq.WQ_EINVAL
    # too small / misaligned workspace are rejected before any upload
    assert _wq.wq_bind(h, dummy, 16, None) == _wq.WQ_ENOSPACE
    assert _wq.wq_bind(h, C.c_void_p(257), 1 << 40, None) == _wq.WQ_ENOSPACE
    assert b"256-byte" in _wq.wq_last_error(h)
    _wq.wq_plan_destroy(h)


def test_first_contraction_offset_limit():
    """Offsets within one i3 plane of the first-contraction buffer are 32-bit
    in the kernels: a patch whose plane holds 2^32 elements or more is
    refused at creation (thin in direction 3, so N_QP itself stays legal)."""
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    p = 2
    # n_qp = 2 n_el + 2p - 1; plane elements n_qp1 n_qp2 (2p+1) 8
    big = open_uniform_knots(p, 5200)    # n_qp = 10403: 10403^2 * 40 > 2^32, N_QP = 10403^2 * 11 < 2^31
    thin = open_uniform_knots(p, p + 2)
    st, _ = make([big, big, thin], p)
    assert st == _wq.WQ_EINVAL
    assert "2^32" in _wq.wq_last_error(None).decode()
    ok = open_uniform_knots(p, 2000)     # 4003^2 * 40 < 2^32
    st, h = make([ok, ok, thin], p)
    assert st == 0
    _wq.wq_plan_destroy(h)


def test_plane_patch_has_no_first_contraction_limit():
    """Plane patches have no first-contraction buffer, so only the N_DOF and
    N_QP limits apply: a plane whose n_qp1 n_qp2 8 reaches 2^32 is accepted."""
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    p = 2
    kn = open_uniform_knots(p, 12000)    # n_qp = 24003: 24003^2 * 8 > 2^32, N_QP = 24003^2 < 2^31
    st, h = make([kn, kn], p)
    assert st == 0, _wq.wq_last_error(None)
    _wq.wq_plan_destroy(h)


def test_static_scratch_size_matches_header():
    import re
    from paper_1605_01238_amd import _wq
    txt = open(os.path.join(ROOT, "include", "wq.h")).read()
    m = re.search(r"#define WQ_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m, "WQ_STATIC_SCRATCH_BYTES not found in wq.h"
    assert int(m.group(1)) << int(m.group(2)) == _wq.WQ_STATIC_SCRATCH_BYTES


def test_batch_host_calls_without_device():
    """wq_batch_create / wq_batch_sizes are host only: classes by (p, d,
    precision), repeated or null plans refused, unbound batches refused."""
    from paper_1605_01238_amd import _wq
    from workloads import open_uniform_knots
    hs = []
    for p, prec in ((2, 0), (3, 0), (2, 0), (2, 1)):
        st, h = make([open_uniform_knots(p, 6)] * 3, p, prec=prec)
        assert st == 0
        hs.append(h)
    arr = (C.c_void_p * 4)(*[h.value for h in hs])
    b = C.c_void_p()
    assert _wq.wq_batch_create(4, arr, C.byref(b)) == 0
    nb, nc = C.c_size_t(), C.c_int()
    assert _wq.wq_batch_sizes(b, C.byref(nb), C.byref(nc)) == 0
    assert nc.value == 3 and nb.value > 0
    info = (C.c_int * 6)()
    assert _wq.wq_batch_schedule(b, 0, info) == 0 and list(info)[:4] == [2, 3, 0, 2]
    assert _wq.wq_batch_schedule(b, 3, info) == _wq.WQ_EINVAL
    assert _wq.wq_batch_assemble(b, 3, 0, None) == _wq.WQ_ESTATE
    assert b"not bound" in _wq.wq_batch_last_error(b)
    _wq.wq_batch_destroy(b)
    rep = (C.c_void_p * 2)(hs[0].value, hs[0].value)
    assert _wq.wq_batch_create(2, rep, C.byref(b)) == _wq.WQ_EINVAL
    assert _wq.wq_batch_create(0, arr, C.byref(b)) == _wq.WQ_EINVAL
    for h in hs:
        _wq.wq_plan_destroy(h)


def test_strip_q2_window_bound():
    """The strip kernel of plane patches stages, per strip of K consecutive
    rows i2, the union of their point sets Q_i2 (Section 4, Remark 4.1
    layout) in a tile sized for 2K + 4p - 1 points.  Checked here on the
    oracle's exact point sets for every K the kernel can take."""
    from oracle.rules import point_set, quadrature_points
    from oracle.splines import exact_knots
    from workloads import open_uniform_knots, random_open_knots
    for p in range(2, 7):
        for nel in (p + 2, p + 3, 2 * p + 3, 23):
            for kn in (open_uniform_knots(p, nel), random_open_knots(p, nel, seed=nel)):
                knots = exact_knots(kn)
                pts = quadrature_points(knots, p)
                n = len(knots) - p - 1
                sets = [point_set(knots, p, pts, i) for i in range(n)]
                for K in range(1, 64 // (2 * p + 1) + 1):
                    for a in range(0, n, K):
                        window = set().union(*sets[a:a + K])
                        assert max(window) - min(window) + 1 <= 2 * K + 4 * p - 1, (p, nel, K, a)
                        assert len(window) == max(window) - min(window) + 1   # contiguous
