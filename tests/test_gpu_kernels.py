"""Kernel-level parity of the HIP building blocks (complex GEMM on MFMA, batched LU
solve, slice eigensolver) against NumPy/LAPACK in FP64."""
import numpy as np
import pytest
import torch

from gpu_common import dev, to_dev

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def lib():
    import paper_1504_01462_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _op(x, op):
    return x if op == 0 else (x.T if op == 1 else x.conj().T)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (16, 16, 4), (37, 37, 37), (64, 64, 16), (65, 63, 17),
                                   (130, 200, 70), (300, 300, 300), (5, 700, 3)])
@pytest.mark.parametrize("ops", [(0, 0), (0, 1), (2, 0), (1, 2)])
def test_gemm_fp64(lib, ctx, m, n, k, ops):
    rng = np.random.default_rng(m * 1000 + n + k)
    op_a, op_b = ops
    a = _rand(rng, (m, k) if op_a == 0 else (k, m))
    b = _rand(rng, (k, n) if op_b == 0 else (n, k))
    c0 = _rand(rng, (m, n))
    alpha, beta = 0.7 - 0.2j, -0.3 + 1.1j
    ref = alpha * (_op(a, op_a) @ _op(b, op_b)) + beta * c0
    c = to_dev(c0)
    lib.ms_debug_gemm(ctx, to_dev(a), to_dev(b), c, op_a, op_b, alpha, beta, "fp64")
    ctx.sync()
    err = np.max(np.abs(c.cpu().numpy() - ref))
    assert err <= 1e-14 * (k + 4) * 4.0, err


@pytest.mark.parametrize("m,n,k", [(37, 37, 37), (130, 200, 70), (300, 300, 300)])
def test_gemm_fp32(lib, ctx, m, n, k):
    rng = np.random.default_rng(7 + m)
    a = _rand(rng, (m, k)).astype(np.complex64)
    b = _rand(rng, (k, n)).astype(np.complex64)
    ref = a.astype(np.complex128) @ b.astype(np.complex128)
    c = lib.ms_debug_gemm(ctx, to_dev(a), to_dev(b), prec="fp32")
    ctx.sync()
    err = np.max(np.abs(c.cpu().numpy() - ref))
    # FP32 products, FP32 accumulation of k terms of size ~|a||b| ~ 2
    assert err <= 6e-8 * 4 * k * 2, err


def _iface_ref(a, o, kp, kq):
    """W[b] = A[b] [C- | C+ with zero diagonal], C-+[m][j] = O[j][m] (kp[j] -+ kq[m]) in FP64."""
    out = []
    for b in range(a.shape[0]):
        cm = o.T * (kp[b][None, :] - kq[b][:, None])
        cp = o.T * (kp[b][None, :] + kq[b][:, None])
        np.fill_diagonal(cp, 0.0)
        out.append(a[b] @ np.hstack([cm, cp]))
    return np.stack(out)


@pytest.mark.parametrize("n,batch", [(1, 1), (7, 3), (37, 2), (64, 2), (65, 3), (130, 2), (300, 4), (1200, 2)])
def test_iface_product_fp64(lib, ctx, n, batch):
    """The fold's interface product with its generated B operand (ragged tile tails), against
    NumPy in FP64."""
    rng = np.random.default_rng(n + 17 * batch)
    a = _rand(rng, (batch, n, n))
    o = _rand(rng, (n, n)) / np.sqrt(n)
    kp = _rand(rng, (batch, n))
    kq = _rand(rng, (batch, n))
    ref = _iface_ref(a, o, kp, kq)
    w = lib.ms_debug_iface_product(ctx, to_dev(a), to_dev(o), to_dev(kp), to_dev(kq), "fp64")
    ctx.sync()
    err = np.max(np.abs(w.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 1e-14 * np.sqrt(n) + 1e-15, err


@pytest.mark.parametrize("n,batch,prec", [(7, 2, "fp64"), (65, 3, "fp64"), (300, 2, "fp64"), (130, 2, "fp32")])
def test_iface_fused_epilogue(lib, ctx, n, batch, prec):
    """The interface product with the fold's epilogue fused into its tile epilogue:
    [C+ + A C- | C- + A C+' + rho_ij C+_jj] against NumPy (rho_ij = P_i kq_i Y_ij P_j / kq_j)."""
    rng = np.random.default_rng(n + 3 * batch)
    a = _rand(rng, (batch, n, n))
    o = _rand(rng, (n, n)) / np.sqrt(n)
    kp = _rand(rng, (batch, n))
    kq = _rand(rng, (batch, n)) + 1.5
    y = _rand(rng, (batch, n, n))
    pq = np.exp(1j * _rand(rng, (batch, n)))
    if prec == "fp32":
        a = a.astype(np.complex64)
    ref = []
    for b in range(batch):
        cm = o.T * (kp[b][None, :] - kq[b][:, None])
        cp = o.T * (kp[b][None, :] + kq[b][:, None])
        cpo = cp.copy()
        np.fill_diagonal(cpo, 0.0)
        rho = (pq[b] * kq[b])[:, None] * y[b] * (pq[b] / kq[b])[None, :]
        ab = a[b].astype(np.complex128)
        ref.append(np.hstack([cp + ab @ cm, cm + ab @ cpo + rho * np.diag(cp)[None, :]]))
    ref = np.stack(ref)
    m = lib.ms_debug_iface_fused(ctx, to_dev(a), to_dev(o), to_dev(kp), to_dev(kq), to_dev(y), to_dev(pq), prec)
    ctx.sync()
    err = np.max(np.abs(m.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= (1e-14 * np.sqrt(n) + 1e-15 if prec == "fp64" else 6e-8 * 8 * np.sqrt(n)), err


@pytest.mark.parametrize("n,batch", [(37, 2), (130, 3), (1200, 2)])
def test_iface_product_fp32(lib, ctx, n, batch):
    """FP32 form: A complex64, B generated in FP64 and rounded when staged, FP32 accumulation."""
    rng = np.random.default_rng(n + 5)
    a = _rand(rng, (batch, n, n)).astype(np.complex64)
    o = _rand(rng, (n, n)) / np.sqrt(n)
    kp = _rand(rng, (batch, n))
    kq = _rand(rng, (batch, n))
    ref = _iface_ref(a.astype(np.complex128), o, kp, kq)
    w = lib.ms_debug_iface_product(ctx, to_dev(a), to_dev(o), to_dev(kp), to_dev(kq), "fp32")
    ctx.sync()
    err = np.max(np.abs(w.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err <= 6e-8 * 8 * np.sqrt(n), err


@pytest.mark.parametrize("n,nrhs,batch", [(1, 1, 2), (5, 3, 3), (16, 16, 2), (17, 13, 2), (37, 74, 3),
                                          (100, 64, 2), (128, 7, 2), (300, 313, 2), (513, 70, 1), (1030, 20, 1)])
def test_lu_solve(lib, ctx, n, nrhs, batch):
    rng = np.random.default_rng(n + nrhs)
    a = _rand(rng, (batch, n, n))
    a[:, np.arange(n), np.arange(n)] *= 1e-3          # force pivoting
    b = _rand(rng, (batch, n, nrhs))
    aug = to_dev(np.concatenate([a, b], axis=2))
    x, st = lib.ms_debug_lu_solve(ctx, aug, n)
    ctx.sync()
    assert np.all(st.cpu().numpy() == 0)
    x = x.cpu().numpy()
    for i in range(batch):
        ref = np.linalg.solve(a[i], b[i])
        res = np.linalg.norm(a[i] @ x[i] - b[i]) / (np.linalg.norm(a[i]) * np.linalg.norm(x[i]))
        assert res < 1e-14 * max(1.0, np.sqrt(n)), res
        cond = np.linalg.cond(a[i])
        assert np.max(np.abs(x[i] - ref)) <= 1e-14 * cond * max(1.0, np.max(np.abs(ref))) * n


def test_lu_singular_flag(lib, ctx):
    n = 20
    rng = np.random.default_rng(3)
    a = _rand(rng, (2, n, n))
    a[1, :, 7] = 0.0                                   # exactly singular second matrix
    aug = to_dev(np.concatenate([a, _rand(rng, (2, n, 2))], axis=2))
    _, st = lib.ms_debug_lu_solve(ctx, aug, n)
    ctx.sync()
    st = st.cpu().numpy()
    assert st[0] == 0 and st[1] == lib.MS_ERR_SINGULAR


def _gershgorin_shift(h):
    off = np.sum(np.abs(h), axis=1) - np.abs(np.diag(h))
    lo = np.min(np.real(np.diag(h)) - off)
    return max(0.0, -lo) + 1.0


@pytest.mark.parametrize("n,batch", [(1, 2), (7, 3), (16, 2), (33, 2), (37, 3), (65, 2), (300, 2)])
def test_eigh(lib, ctx, n, batch):
    rng = np.random.default_rng(100 + n)
    h = _rand(rng, (batch, n, n))
    h = 0.5 * (h + np.conj(np.transpose(h, (0, 2, 1))))
    if n >= 7:   # an exactly degenerate block and a decoupled diagonal entry
        h[0, :3, :] = 0.0
        h[0, :, :3] = 0.0
        h[0, 0, 0] = h[0, 1, 1] = h[0, 2, 2] = 0.25
    shift = np.array([_gershgorin_shift(x) for x in h])
    eps, u = lib.ms_debug_eigh(ctx, to_dev(h), to_dev(shift))
    ctx.sync()
    eps, u = eps.cpu().numpy(), u.cpu().numpy()
    for i in range(batch):
        ref = np.linalg.eigvalsh(h[i])
        scale = max(1.0, np.linalg.norm(h[i], 2))
        assert np.max(np.abs(eps[i] - ref)) < 1e-12 * scale
        assert np.linalg.norm(h[i] @ u[i] - u[i] * eps[i]) < 1e-12 * scale * np.sqrt(n)
        assert np.max(np.abs(u[i].conj().T @ u[i] - np.eye(n))) < 1e-12


def _qz_check(lib, ctx, a, b, tol=1e-11):
    """QZ eigenpairs against LAPACK (scipy.linalg.eig): residuals of every pair, and the finite
    eigenvalues matched one to one."""
    import scipy.linalg as sla
    al, be, x, st = (t.cpu().numpy() for t in lib.ms_debug_qz(ctx, to_dev(a), to_dev(b)))
    ctx.sync()
    assert np.all(st == 0)
    for i in range(a.shape[0]):
        na, nb = np.linalg.norm(a[i]), np.linalg.norm(b[i])
        res = np.linalg.norm(be[i][None, :] * (a[i] @ x[i]) - al[i][None, :] * (b[i] @ x[i]), axis=0)
        scale = np.abs(be[i]) * na + np.abs(al[i]) * nb
        assert np.max(res / scale) < tol, np.max(res / scale)
        assert np.allclose(np.linalg.norm(x[i], axis=0), 1.0, atol=1e-12)
        ref = sla.eigvals(a[i], b[i])
        fin = np.abs(be[i]) > 1e-8 * (np.abs(al[i]) + 1e-300)
        got = list(al[i][fin] / be[i][fin])
        for w in ref[np.isfinite(ref) & (np.abs(ref) < 1e6)]:
            d = [abs(g - w) / max(1.0, abs(w)) for g in got]
            k = int(np.argmin(d))
            assert d[k] < 1e-9, (w, got[k])
            got.pop(k)
    return al, be, x


@pytest.mark.parametrize("n,batch", [(2, 3), (5, 2), (16, 2), (37, 3), (64, 2), (130, 1)])
def test_qz_random_pencils(lib, ctx, n, batch):
    rng = np.random.default_rng(11 + n)
    _qz_check(lib, ctx, _rand(rng, (batch, n, n)), _rand(rng, (batch, n, n)))


def test_qz_singular_b_infinite_eigenvalues(lib, ctx):
    """B of rank n - 3: three infinite eigenvalues (beta = 0) deflated by chasing the zeros of
    B's diagonal; the finite ones match LAPACK."""
    rng = np.random.default_rng(5)
    n = 24
    a = _rand(rng, (2, n, n))
    b = _rand(rng, (2, n, n - 3)) @ _rand(rng, (2, n - 3, n))
    al, be, _ = _qz_check(lib, ctx, a, b, tol=1e-10)
    for i in range(2):
        assert np.sum(np.abs(be[i]) < 1e-9 * np.abs(al[i])) == 3
