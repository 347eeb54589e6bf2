"""Single-kernel checks on the GPU through the test-only harness library.

The block product is compared with a plain product computed on the CPU
(complex128 numpy); the blocked LU with partial pivoting and its two block
triangular solves with ``numpy.linalg.solve``; the adjoint formation kernel
with the element-wise fill and numpy.
"""
import ctypes as C
import os

import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu

KT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                  "paper_2609_37058_amd", "librgf_ktest.so")


@pytest.fixture(scope="module")
def kt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = C.CDLL(KT)
    lib.rgf_ktest_gemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_double, C.c_int]
    lib.rgf_ktest_lu.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]
    lib.rgf_ktest_form_ct.argtypes = [C.c_int] * 5 + [C.c_void_p] * 3 + [C.c_double, C.c_void_p, C.c_void_p]
    lib.rgf_ktest_gj.argtypes = [C.c_int] * 3 + [C.c_void_p] * 6
    lib.rgf_ktest_set_small_k.argtypes = [C.c_int]
    lib.rgf_ktest_set_lookahead.argtypes = [C.c_int]
    lib.rgf_ktest_set_exact_u.argtypes = [C.c_int]
    return lib


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("prec,tile", [(0, 64), (1, 64), (1, 128), (0, 128)])
@pytest.mark.parametrize("rows,cols,K,batch", [(64, 64, 16, 1), (128, 64, 64, 3), (128, 256, 48, 2),
                                               (192, 320, 32, 2), (320, 192, 80, 3), (64, 448, 64, 2),
                                               (192, 192, 256, 2), (64, 320, 144, 2)])
def test_gemm_matches_numpy(kt, prec, tile, rows, cols, K, batch):
    """Shapes that are multiples of 64 but not of 128 run on 128-wide tiles that overhang the matrix;
    K <= 128 with 128-wide tiles takes the short-K tiles, the last two shapes the 8-wavefront ones."""
    import torch
    rng = np.random.default_rng(rows + cols + K + batch)
    A = _rand(rng, (batch, rows, K))
    B = _rand(rng, (batch, K, cols))
    C0 = _rand(rng, (batch, rows, cols))
    ta, tb, tc = (torch.as_tensor(x).cuda() for x in (A, B, C0))
    log(f"[kernel] gemm prec={prec} tile={tile} {rows}x{cols}x{K} b={batch}")
    rc = kt.rgf_ktest_gemm(prec, tile, rows, cols, K, batch, ta.data_ptr(), tb.data_ptr(), tc.data_ptr(),
                           -1.0, 1)
    assert rc == 0
    got = tc.cpu().numpy()
    ref = C0 - A @ B
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    log(f"[kernel] gemm rel err {err:.2e}")
    assert err < (1e-14 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("rows,cols,K,batch", [(64, 1024, 64, 3), (960, 960, 64, 2), (896, 896, 128, 2),
                                               (192, 320, 16, 2), (128, 64, 112, 3)])
def test_short_k_tiles_bitwise_equal_to_wide_tiles(kt, prec, rows, cols, K, batch):
    """The short-K tiles (4 wavefronts, 8-column stages) sum every output's K terms in the same
    order as the 8-wavefront tiles, so the two give identical bits."""
    import torch
    rng = np.random.default_rng(7 * rows + cols + K)
    A = _rand(rng, (batch, rows, K))
    B = _rand(rng, (batch, K, cols))
    C0 = _rand(rng, (batch, rows, cols))
    ta, tb = (torch.as_tensor(x).cuda() for x in (A, B))
    out = []
    prev = kt.rgf_ktest_set_small_k(128)
    try:
        for k in (128, 0):
            kt.rgf_ktest_set_small_k(k)
            tc = torch.as_tensor(C0).cuda()
            log(f"[kernel] short-K={k} prec={prec} {rows}x{cols}x{K} b={batch}")
            assert kt.rgf_ktest_gemm(prec, 128, rows, cols, K, batch, ta.data_ptr(), tb.data_ptr(), tc.data_ptr(),
                                     -1.0, 1) == 0
            out.append(tc.cpu().numpy())
    finally:
        kt.rgf_ktest_set_small_k(prev)
    assert np.array_equal(out[0], out[1])
    ref = C0 - A @ B
    assert np.max(np.abs(out[0] - ref)) / np.max(np.abs(ref)) < (1e-14 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("Mp,batch", [(320, 3), (512, 2), (1024, 2), (1152, 2)])
def test_lu_lookahead_bitwise_equal(kt, prec, Mp, batch):
    """The look-ahead factorisation (far columns updated on a side stream, candidate lists
    alternating between pairs of panels) runs the same products on the same data as the plain
    one, split at other column boundaries: identical bits, and the solve still matches numpy."""
    import torch
    rng = np.random.default_rng(Mp + 3 * batch)
    Bm = _rand(rng, (batch, Mp, Mp)) * np.exp(rng.uniform(-3, 3, size=(batch, Mp, 1)))
    R = _rand(rng, (batch, Mp, 64))
    tr = torch.as_tensor(np.ascontiguousarray(R)).cuda()
    outs = []
    prev = kt.rgf_ktest_set_lookahead(1)
    try:
        for la in (1, 0):
            kt.rgf_ktest_set_lookahead(la)
            tb = torch.as_tensor(np.ascontiguousarray(Bm)).cuda()
            X = torch.zeros((batch, Mp, 64), dtype=torch.complex128, device="cuda")
            perm = np.zeros((batch, Mp), np.int32)
            sing = np.zeros(batch, np.int32)
            log(f"[kernel] lu look-ahead={la} prec={prec} Mp={Mp} b={batch}")
            assert kt.rgf_ktest_lu(prec, Mp, 64, batch, tb.data_ptr(), tr.data_ptr(), X.data_ptr(),
                                   perm.ctypes.data, sing.ctypes.data) == 0
            outs.append((X.cpu().numpy(), perm.copy(), sing.copy()))
    finally:
        kt.rgf_ktest_set_lookahead(prev)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert np.all(outs[0][2] == 0)
    ref = np.linalg.solve(Bm, R)
    err = np.max(np.abs(outs[0][0] - ref)) / np.max(np.abs(ref))
    # the bar of test_lu_solve_matches_numpy_solve (FP32: the error grows with the order)
    assert err < (1e-11 if prec == 0 else 1e-3 * max(1.0, Mp / 512))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("Mp,nrhs,batch", [(64, 64, 2), (128, 128, 3), (192, 384, 2), (256, 256, 1), (512, 128, 2),
                                           (576, 64, 2), (1024, 128, 2), (1152, 64, 2), (2048, 64, 1)])
def test_lu_solve_matches_numpy_solve(kt, prec, Mp, nrhs, batch):
    import torch
    rng = np.random.default_rng(Mp + nrhs)
    Bm = _rand(rng, (batch, Mp, Mp))
    # rows scaled so that partial pivoting must reorder them
    Bm *= np.exp(rng.uniform(-3, 3, size=(batch, Mp, 1)))
    R = _rand(rng, (batch, Mp, nrhs))
    tb = torch.as_tensor(np.ascontiguousarray(Bm)).cuda()
    tr = torch.as_tensor(np.ascontiguousarray(R)).cuda()
    X = torch.zeros((batch, Mp, nrhs), dtype=torch.complex128, device="cuda")
    perm = np.zeros((batch, Mp), np.int32)
    sing = np.zeros(batch, np.int32)
    log(f"[kernel] lu prec={prec} Mp={Mp} nrhs={nrhs} b={batch}")
    rc = kt.rgf_ktest_lu(prec, Mp, nrhs, batch, tb.data_ptr(), tr.data_ptr(), X.data_ptr(), perm.ctypes.data,
                         sing.ctypes.data)
    assert rc == 0
    got = X.cpu().numpy()
    ref = np.linalg.solve(Bm, R)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    log(f"[kernel] lu rel err {err:.2e}")
    assert all(sorted(p) == list(range(Mp)) for p in perm)
    assert np.all(sing == 0)
    # FP32 trailing updates and solves: the error grows with the order of these row-scaled random systems
    assert err < (1e-11 if prec == 0 else 1e-3 * max(1.0, Mp / 512))


@pytest.mark.parametrize("Mp,nrhs,batch,graded", [(128, 128, 2, False), (512, 320, 2, False), (1024, 128, 1, False),
                                                  (256, 256, 2, True), (1024, 64, 1, True)])
def test_lu_solve_with_exact_u_blocks(kt, Mp, nrhs, batch, graded):
    """The decimation's solve: the panel kernel keeps U's 64 x 64 diagonal blocks and the solve
    back-substitutes with them instead of applying their inverses.  On row-scaled random systems
    it matches numpy's solve like the default path; on column-graded ones (columns scaled over
    twelve decades, so U's diagonal blocks are ill-conditioned) its backward error stays at
    rounding level."""
    import torch
    rng = np.random.default_rng(7 * Mp + nrhs)
    Bm = _rand(rng, (batch, Mp, Mp))
    if graded:
        Bm *= 10.0 ** rng.uniform(-12, 0, size=(batch, 1, Mp))
    else:
        Bm *= np.exp(rng.uniform(-3, 3, size=(batch, Mp, 1)))
    R = _rand(rng, (batch, Mp, nrhs))
    tr = torch.as_tensor(np.ascontiguousarray(R)).cuda()
    tb = torch.as_tensor(np.ascontiguousarray(Bm)).cuda()
    X = torch.zeros((batch, Mp, nrhs), dtype=torch.complex128, device="cuda")
    perm = np.zeros((batch, Mp), np.int32)
    sing = np.zeros(batch, np.int32)
    log(f"[kernel] lu exact U blocks Mp={Mp} nrhs={nrhs} b={batch} graded={graded}")
    prev = kt.rgf_ktest_set_exact_u(1)
    try:
        assert kt.rgf_ktest_lu(0, Mp, nrhs, batch, tb.data_ptr(), tr.data_ptr(), X.data_ptr(), perm.ctypes.data,
                               sing.ctypes.data) == 0
    finally:
        kt.rgf_ktest_set_exact_u(prev)
    got = X.cpu().numpy()
    assert np.all(sing == 0)
    if graded:
        res = np.einsum("bij,bjk->bik", Bm, got) - R
        back = max(np.linalg.norm(res[b]) / (np.linalg.norm(Bm[b]) * np.linalg.norm(got[b]) + np.linalg.norm(R[b]))
                   for b in range(batch))
        log(f"[kernel] lu exact U blocks backward error {back:.2e}")
        assert back < 1e-13
    else:
        ref = np.linalg.solve(Bm, R)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        log(f"[kernel] lu exact U blocks rel err {err:.2e}")
        assert err < 1e-11


@pytest.mark.parametrize("M,Mp,batch,groups,pad", [(64, 64, 1, 1, 0), (100, 128, 13, 1, 0), (130, 192, 9, 3, 1),
                                                   (1024, 1024, 3, 3, 0), (33, 64, 17, 17, 1)])
def test_adjoint_formation_kernel(kt, M, Mp, batch, groups, pad):
    """z_b S^+ - H^+ written by the tiled kernel equals the element-wise fill bitwise and the
    definition (numpy) to rounding; the padding is zero (identity on the diagonal with pad)."""
    import torch
    rng = np.random.default_rng(M + batch)
    H = _rand(rng, (groups, M, M))
    S = _rand(rng, (groups, M, M))
    E = np.linspace(-1.0, 1.0, batch)
    eta = 1e-3
    th, ts = torch.as_tensor(H).cuda(), torch.as_tensor(S).cuda()
    te = torch.as_tensor(E).cuda()
    oc = torch.full((batch, Mp, Mp), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
    of = torch.full((batch, Mp, Mp), complex(-7.0, 7.0), dtype=torch.complex128, device="cuda")
    rc = kt.rgf_ktest_form_ct(M, Mp, batch, groups, pad, th.data_ptr(), ts.data_ptr(), te.data_ptr(), eta,
                              oc.data_ptr(), of.data_ptr())
    assert rc == 0
    oc, of = oc.cpu().numpy(), of.cpu().numpy()
    assert np.array_equal(oc.view(np.float64), of.view(np.float64))
    per = -(-batch // groups)
    for b in range(batch):
        g = b // per
        ref = np.zeros((Mp, Mp), dtype=np.complex128)
        if pad:
            ref[np.arange(M, Mp), np.arange(M, Mp)] = 1.0
        ref[:M, :M] = (E[b] + 1j * eta) * S[g].conj().T - H[g].conj().T
        assert np.allclose(oc[b], ref, rtol=0, atol=1e-14 * (1 + np.abs(ref).max()))
        assert np.array_equal(oc[b][M:, :], ref[M:, :]) and np.array_equal(oc[b][:, M:], ref[:, M:])


@pytest.mark.parametrize("Mp,rhs,batch", [(64, 1, 3), (64, 2, 2), (128, 1, 3), (128, 2, 2), (192, 1, 2),
                                          (256, 1, 3), (256, 2, 2)])
def test_fused_factor_solve_matches_numpy_solve(kt, Mp, rhs, batch):
    """The fused Gauss-Jordan factor-and-solve (one workgroup per entry) against numpy.linalg.solve,
    with rows scaled so that partial pivoting must reorder them, nrhs = Mp and 2 Mp; the pivot rows
    are a permutation; entry 1 is skipped and must come back untouched."""
    import torch
    nrhs = rhs * Mp
    rng = np.random.default_rng(7 * Mp + nrhs)
    Bm = _rand(rng, (batch, Mp, Mp))
    Bm *= np.exp(rng.uniform(-3, 3, size=(batch, Mp, 1)))
    R = _rand(rng, (batch, Mp, nrhs))
    tb = torch.as_tensor(np.ascontiguousarray(Bm)).cuda()
    ty = torch.as_tensor(np.ascontiguousarray(R)).cuda()
    X = torch.zeros((batch, Mp, nrhs), dtype=torch.complex128, device="cuda")
    perm = np.zeros((batch, Mp), np.int32)
    sing = np.zeros(batch, np.int32)
    skip = np.zeros(batch, np.int32)
    skip[1] = 1
    log(f"[kernel] fused gj Mp={Mp} nrhs={nrhs} b={batch}")
    rc = kt.rgf_ktest_gj(Mp, nrhs, batch, tb.data_ptr(), ty.data_ptr(), X.data_ptr(), skip.ctypes.data,
                         perm.ctypes.data, sing.ctypes.data)
    assert rc == 0
    got = X.cpu().numpy()
    ref = np.linalg.solve(Bm, R)
    for b in range(batch):
        if b == 1:
            assert np.array_equal(tb[1].cpu().numpy(), Bm[1]) and np.array_equal(ty[1].cpu().numpy(), R[1])
            continue
        err = np.max(np.abs(got[b] - ref[b])) / np.max(np.abs(ref[b]))
        log(f"[kernel]   entry {b}: rel err {err:.2e}")
        assert err < 1e-11
        assert sorted(perm[b].tolist()) == list(range(Mp))
    assert np.all(sing == 0)


def test_fused_factor_solve_flags_exact_zero_pivot(kt):
    """An all-zero column makes an exactly zero pivot: the entry's singular code is set (and only
    that entry's); the kernel finishes normally."""
    import torch
    Mp, nrhs, batch = 128, 128, 2
    rng = np.random.default_rng(3)
    Bm = _rand(rng, (batch, Mp, Mp))
    Bm[0, :, 40] = 0.0
    R = _rand(rng, (batch, Mp, nrhs))
    tb = torch.as_tensor(np.ascontiguousarray(Bm)).cuda()
    ty = torch.as_tensor(np.ascontiguousarray(R)).cuda()
    X = torch.zeros((batch, Mp, nrhs), dtype=torch.complex128, device="cuda")
    sing = np.zeros(batch, np.int32)
    rc = kt.rgf_ktest_gj(Mp, nrhs, batch, tb.data_ptr(), ty.data_ptr(), X.data_ptr(), None, None, sing.ctypes.data)
    assert rc == 0
    assert sing[0] == 7 and sing[1] == 0
    got = X.cpu().numpy()
    assert np.max(np.abs(got[1] - np.linalg.solve(Bm[1], R[1]))) < 1e-10 * np.max(np.abs(got[1]))
