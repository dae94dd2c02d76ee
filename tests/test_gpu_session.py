"""The input session shaped like the paper's library interface (App. B): the tiny workload fed
through rpa_set_* calls gives E_c bitwise equal to the direct path (build_green_tau,
build_chi0_tau, chi0_tau_to_omega, chi0_R_to_q, rpa_correlation_energy on the same data and the
same block order), and within 1e-10 Ha/atom of the FP64 oracle; irreducible q points with weights
give the weighted per-q terms; missing or inconsistent inputs are rejected with their codes."""
import numpy as np
import pytest

from tests._util import cfg

pytestmark = pytest.mark.gpu


def sorted_blocks(inp):
    """LRI blocks in (I, K, R) order, the order the session keeps them in."""
    b = inp.blocks
    keys = [(int(b.I[i]), int(b.K[i]), *[int(x) for x in b.R[i]]) for i in range(len(b.I))]
    return sorted(range(len(b.I)), key=lambda i: keys[i])


def feed(sess, inp, ibz=None, pair_coulomb=True):
    nk, nb = inp.eps.shape
    natoms = inp.natoms
    sess.set_dimension(1, nk, nb, nb, natoms)
    wg = np.zeros((nk, nb))
    wg[:, :inp.nocc] = 2.0 / nk
    sess.set_wg_ekb_efermi(1, nk, nb, wg, inp.eps, inp.mu)
    for k in range(nk):
        c = inp.wfc[k]                                   # c_{i n} at [i][n]
        sess.set_ao_basis_wfc(0, k, np.ascontiguousarray(c.real.T), np.ascontiguousarray(c.imag.T))
    # lattice 2 pi I: the fractional coordinates k . a / (2 pi) of the mesh come out exactly
    sess.set_latvec_and_G(2 * np.pi * np.eye(3), np.eye(3))
    sess.set_kgrids_kvec_tot(*inp.cell.mesh, inp.kfrac)
    if ibz is not None:
        sess.set_ibz2bz_index_and_weight(*ibz)
    b = inp.blocks
    for i in sorted_blocks(inp):
        I, K = int(b.I[i]), int(b.K[i])
        sess.set_ao_basis_aux(I, K, inp.nao[I], inp.nao[K], inp.naux[I], b.R[i], b.block(i, inp.naux, inp.nao))
    qs = ibz[0] if ibz is not None else range(nk)
    for iq, k in enumerate(qs):
        v = inp.vq[k]
        if pair_coulomb:
            for I in range(natoms):
                mu = slice(inp.aux_off[I], inp.aux_off[I] + inp.naux[I])
                for J in range(natoms):
                    nu = slice(inp.aux_off[J], inp.aux_off[J] + inp.naux[J])
                    sess.set_aux_bare_coulomb_k_atom_pair(iq, I, J, inp.naux[I], inp.naux[J], v[mu, nu].real,
                                                          v[mu, nu].imag)
        else:
            N = inp.nauxtot
            h = N // 2
            for (m0, m1, n0, n1) in ((0, h, 0, N), (h, N, 0, h), (h, N, h, N)):
                sess.set_aux_bare_coulomb_k_2D_block(iq, N, m0, m1, n0, n1, v[m0:m1, n0:n1].real,
                                                     v[m0:m1, n0:n1].imag)
    sess.set_time_freq_grids(inp.tau, inp.womega, inp.gamma_cos)


def direct_path(ctx, inp, precision="fp64"):
    """The same data through the compute calls, G from the eigenpairs on the GPU, blocks sorted."""
    import torch
    from paper_2407_19930_amd import (Plan, build_chi0_tau, build_green_tau, chi0_R_to_q, chi0_tau_to_omega,
                                      rpa_correlation_energy, rpa_ec_workspace_size, rpa_green_workspace_size)
    nk, nb = inp.eps.shape
    order = sorted_blocks(inp)
    b = inp.blocks
    Cs = [b.block(i, inp.naux, inp.nao).ravel() for i in order]
    off = np.cumsum([0] + [c.size for c in Cs[:-1]])
    C = torch.from_numpy(np.concatenate(Cs)).cuda()
    plan = Plan(ctx, inp.nao, inp.naux, inp.cell.mesh, b.I[order], b.K[order], b.R[order], off, inp.ntau, precision)
    eps = torch.from_numpy(np.ascontiguousarray(inp.eps)).cuda()
    wfc = torch.from_numpy(np.ascontiguousarray(inp.wfc)).cuda()
    gws = torch.empty(rpa_green_workspace_size(nk, nb, inp.nocc), dtype=torch.uint8, device="cuda")
    Go = torch.empty((inp.ntau, inp.nR, nb, nb), dtype=torch.float64, device="cuda")
    Gu = torch.empty_like(Go)
    build_green_tau(ctx, eps, wfc, inp.nocc, inp.mu, inp.tau, inp.cell.mesh, inp.kfrac, gws, Go, Gu)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    N, nR, nt, nq = inp.nauxtot, inp.nR, inp.ntau, len(inp.kfrac)
    chi = torch.empty((nt, nR, N, N), dtype=torch.float64, device="cuda")
    build_chi0_tau(plan, 2.0, Go, Gu, C, ws, chi)
    chi_w = torch.empty((nt, nR, N, N), dtype=torch.float64, device="cuda")
    chi0_tau_to_omega(ctx, inp.gamma_cos, chi, chi_w)
    chi_q = torch.empty((nt, nq, N, N), dtype=torch.complex128, device="cuda")
    chi0_R_to_q(ctx, inp.cell.mesh, inp.kfrac, chi_w, chi_q)
    ews = torch.empty(rpa_ec_workspace_size(N, nq, nt), dtype=torch.uint8, device="cuda")
    ec, ecq = rpa_correlation_energy(ctx, inp.womega, chi_q, torch.from_numpy(inp.vq).cuda(), ews)
    plan.close()
    return ec, ecq


@pytest.mark.parametrize("pair_coulomb", [True, False])
def test_session_matches_direct_path_bitwise(pair_coulomb):
    from oracle.pipeline import ec_from_chi_tau
    from oracle import chi0 as ochi
    from paper_2407_19930_amd import Context, Session
    inp = cfg(0)
    ctx = Context(0)
    sess = Session(ctx)
    feed(sess, inp, pair_coulomb=pair_coulomb)
    ec, contrib = sess.get_rpa_correlation_energy()
    ec_d, ecq_d = direct_path(ctx, inp)
    print("session E_c %.15g, direct %.15g" % (ec, ec_d), flush=True)
    assert ec == ec_d
    np.testing.assert_allclose(contrib, ecq_d, rtol=0, atol=1e-15 * abs(ec_d))
    assert abs(contrib.sum() - ec) <= 1e-14 * abs(ec)
    ec_ref, _, _ = ec_from_chi_tau(inp, ochi.chi0_alg1(inp))
    assert abs(ec - ec_ref) / inp.natoms <= 1e-10
    sess.close()


def test_session_irreducible_points_and_precision():
    """Irreducible q points (a subset with weights): contribution i = w_i (1/2 pi) sum_k w_k f(q_i)
    = w_i nq Ec_q of the direct path; and the split-BF16 build through the session within the
    mixed-path bar of FP64."""
    from paper_2407_19930_amd import Context, Session
    inp = cfg(0)
    ctx = Context(0)
    nk = len(inp.kfrac)
    ec_d, ecq_d = direct_path(ctx, inp)
    idx = np.array([0, 3, 5, 6], dtype=np.int32)
    w = np.array([1.0, 2.0, 3.0, 2.0])
    sess = Session(ctx)
    feed(sess, inp, ibz=(idx, w))
    ec, contrib = sess.get_rpa_correlation_energy()
    want = (w / w.sum()) * nk * ecq_d[idx]
    np.testing.assert_allclose(contrib, want, rtol=1e-12, atol=0)
    assert abs(ec - want.sum()) <= 1e-12 * abs(ec)
    sess.close()
    sb = Session(ctx)
    sb.set_precision("bf16x3")
    feed(sb, inp)
    ecb, _ = sb.get_rpa_correlation_energy()
    assert abs(ecb - ec_d) / inp.natoms <= 1e-6
    sb.close()


def test_session_errors():
    from paper_2407_19930_amd import Context, RpaError, Session
    from paper_2407_19930_amd.binding import RPA_ERR_ARG, RPA_ERR_SHAPE, RPA_ERR_UNSUPPORTED
    inp = cfg(0)
    ctx = Context(0)
    s = Session(ctx)
    nk, nb = inp.eps.shape
    with pytest.raises(RpaError) as e:
        s.set_dimension(2, nk, nb, nb, inp.natoms)          # spin-polarised
    assert e.value.code == RPA_ERR_UNSUPPORTED
    with pytest.raises(RpaError) as e:
        s.get_rpa_correlation_energy()                      # nothing set
    assert e.value.code == RPA_ERR_SHAPE
    s.set_dimension(1, nk, nb, nb, inp.natoms)
    with pytest.raises(RpaError) as e:
        s.set_kgrids_kvec_tot(3, 3, 3, np.zeros((27, 3)))   # not the k count
    assert e.value.code == RPA_ERR_SHAPE
    with pytest.raises(RpaError) as e:
        s.set_ao_basis_aux(inp.natoms, 0, 1, 1, 1, [0, 0, 0], np.zeros(1))
    assert e.value.code == RPA_ERR_ARG
    with pytest.raises(RpaError) as e:
        s.set_ibz2bz_index_and_weight([0, nk], [1.0, 1.0])
    assert e.value.code == RPA_ERR_ARG
    feed(s, inp)
    # a Coulomb block left out of the last q point
    s.set_ibz2bz_index_and_weight(np.arange(nk, dtype=np.int32), np.ones(nk))
    with pytest.raises(RpaError) as e:
        s.get_rpa_correlation_energy()
    assert e.value.code == RPA_ERR_SHAPE
    s.close()
