"""The energy stage on q points where chi(q, i omega) and v(q) are both real (the real-layout
kernels: real GEMM with 128 x 128 tiles, Cholesky pieces on real row-major matrices) beside q
points that stay complex (chi real with v complex, and both complex), in one call and in batches
that mix them: per-q terms against the oracle's LU log-determinant (Sec. 2, E_c with
Tr ln = ln det) on the same matrices.  n = 1600 spans several GEMM tiles with a ragged last
one, and takes the Cholesky's 8-panel blocks; n = 4160 its 16-panel blocks."""
import numpy as np
import pytest

from oracle.energy import correlation_energy, ec_terms_lu
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _norm2(h):
    """Spectral norm of a Hermitian matrix, with a little margin for the Lanczos tolerance."""
    from scipy.sparse.linalg import eigsh
    return 1.001 * float(np.abs(eigsh(h, k=1, which="LM", return_eigenvectors=False, tol=1e-6)[0]))


def _inputs(n, seed=5):
    """chi[k, q] = -s X X^H / (k + 1) (negative semidefinite), v[q] = Y Y^H + 0.1 I, each scaled
    by its largest eigenvalue in magnitude (Lanczos), so that the norm of chi v stays below 1/2; q = 0: X, Y real; q = 1: X real, Y complex;
    q = 2: both complex."""
    rng = np.random.default_rng(seed)
    nq, nw = 3, 2
    chi = np.empty((nw, nq, n, n), dtype=np.complex128)
    vq = np.empty((nq, n, n), dtype=np.complex128)
    for q in range(nq):
        X = rng.standard_normal((n, n // 2)) + (1j * rng.standard_normal((n, n // 2)) if q == 2 else 0)
        Y = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if q >= 1 else 0)
        c = -(X @ X.conj().T)
        c = 0.5 * (c + c.conj().T)
        v = Y @ Y.conj().T + 0.1 * np.eye(n)
        v = 0.5 * (v + v.conj().T)
        c /= _norm2(c)
        v /= _norm2(v)
        vq[q] = v
        for k in range(nw):
            chi[k, q] = 0.5 * c / (k + 1)
    assert np.all(chi[:, :2].imag == 0) and np.all(vq[0].imag == 0)
    assert np.any(vq[1].imag != 0) and np.any(chi[:, 2].imag != 0)
    return chi, vq, np.array([0.7, 0.3])


def test_real_and_complex_q_points_against_lu():
    import torch
    from paper_2407_19930_amd import Context, rpa_correlation_energy, rpa_ec_workspace_size
    n = 1600
    chi, vq, w = _inputs(n)
    nw, nq = chi.shape[:2]
    f = ec_terms_lu(chi, vq)
    ec_ref, perq_ref = correlation_energy(f, w)
    ctx = Context(0)
    chi_d = torch.from_numpy(chi).cuda()
    v_d = torch.from_numpy(vq).cuda()
    full = rpa_ec_workspace_size(n, nq, nw)
    per_pair = 2 * n * n * 16
    # every (q, omega) pair in one batch; then batches of three that mix real and complex pairs
    for size in (full, full - 3 * per_pair):
        say("case energy real/complex q, n %d, workspace %d bytes" % (n, size))
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        ec, perq = rpa_correlation_energy(ctx, w, chi_d, v_d, ws)
        say("  per q gpu", perq, "oracle LU", perq_ref)
        np.testing.assert_allclose(perq, perq_ref, rtol=1e-10, atol=0)
        assert abs(ec - ec_ref) <= 1e-10 * abs(ec_ref)
        del ws
        torch.cuda.synchronize()


def test_real_q_point_not_positive_definite_is_flagged():
    """chi real and v real with 1 - L^T chi L indefinite: the real Cholesky reports it like the
    complex one (RPA_ERR_NOT_HPD)."""
    import torch
    from paper_2407_19930_amd import Context, RpaError, rpa_correlation_energy, rpa_ec_workspace_size
    from paper_2407_19930_amd.binding import RPA_ERR_NOT_HPD
    n = 300
    chi, vq, w = _inputs(n, seed=7)
    chi = np.ascontiguousarray(chi[:, :1])
    vq = np.ascontiguousarray(vq[:1])
    chi[1, 0] = -chi[1, 0] * 40.0         # positive chi at omega_1: 1 - L^T chi L indefinite
    L = np.linalg.cholesky(vq[0].real)
    assert np.linalg.eigvalsh(np.eye(n) - L.T @ chi[1, 0].real @ L)[0] < 0
    ctx = Context(0)
    ws = torch.empty(rpa_ec_workspace_size(n, 1, 2), dtype=torch.uint8, device="cuda")
    say("case energy real q, indefinite")
    with pytest.raises(RpaError) as e:
        rpa_correlation_energy(ctx, w, torch.from_numpy(chi).cuda(), torch.from_numpy(vq).cuda(), ws)
    assert e.value.code == RPA_ERR_NOT_HPD


def test_real_q_point_sixteen_panel_blocks():
    """One real q point of order 4160 (the Cholesky's 16-panel blocks, a ragged last GEMM tile)
    against the oracle's LU."""
    import torch
    from paper_2407_19930_amd import Context, rpa_correlation_energy, rpa_ec_workspace_size
    n = 4160
    rng = np.random.default_rng(11)
    X = rng.standard_normal((n, n // 2))
    c = -(X @ X.T)
    c /= _norm2(c)
    Y = rng.standard_normal((n, n))
    v = Y @ Y.T + 0.1 * np.eye(n)
    v /= _norm2(v)
    chi = (0.5 * c).astype(np.complex128).reshape(1, 1, n, n)
    vq = v.astype(np.complex128).reshape(1, n, n)
    w = np.array([1.0])
    f = ec_terms_lu(chi, vq)
    ec_ref, _ = correlation_energy(f, w)
    ctx = Context(0)
    ws = torch.empty(rpa_ec_workspace_size(n, 1, 1), dtype=torch.uint8, device="cuda")
    say("case energy real q, n %d" % n)
    ec, _ = rpa_correlation_energy(ctx, w, torch.from_numpy(chi).cuda(), torch.from_numpy(vq).cuda(), ws)
    say("  E_c gpu %.15g oracle LU %.15g" % (ec, ec_ref))
    assert abs(ec - ec_ref) <= 1e-10 * abs(ec_ref)


@pytest.mark.parametrize("keep", [(0,), (2,), (1, 2)])
def test_calls_with_one_kind_of_q_point(keep):
    """Calls whose q points are all real-layout (q 0), all complex (q 2), or complex with a real
    chi (q 1) beside a complex one: the launches of the absent kind are left out, and the per-q
    terms still match the oracle's LU."""
    import torch
    from paper_2407_19930_amd import Context, rpa_correlation_energy, rpa_ec_workspace_size
    n = 300
    chi, vq, w = _inputs(n, seed=13)
    idx = list(keep)
    chi = np.ascontiguousarray(chi[:, idx])
    vq = np.ascontiguousarray(vq[idx])
    f = ec_terms_lu(chi, vq)
    ec_ref, perq_ref = correlation_energy(f, w)
    ctx = Context(0)
    nw, nq = chi.shape[:2]
    ws = torch.empty(rpa_ec_workspace_size(n, nq, nw), dtype=torch.uint8, device="cuda")
    say("case energy, q points", keep)
    ec, perq = rpa_correlation_energy(ctx, w, torch.from_numpy(chi).cuda(), torch.from_numpy(vq).cuda(), ws)
    np.testing.assert_allclose(perq, perq_ref, rtol=1e-10, atol=0)
    assert abs(ec - ec_ref) <= 1e-10 * abs(ec_ref)
