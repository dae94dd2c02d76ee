// Input session in the shape of the paper's library interface (App. B): the host program hands
// over dimensions, band energies and occupations, Bloch eigenvectors, lattice and k mesh, the
// irreducible k points, LRI coefficients per atom pair and the Coulomb matrix per atom pair or 2D
// block; one call then runs the whole path on the GPU (Green's functions from the eigenpairs,
// chi0(R, tau), tau -> i omega, R -> q, E_c) through the library's own entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rpa_mi355x.h"

namespace {

struct AuxBlock {
  int I, J, ni, nj, na;
  int R[3];
  std::vector<double> C;      // [na][ni][nj]
};

}  // namespace

struct rpa_session {
  rpa_ctx *ctx = nullptr;
  std::string err;
  int precision = RPA_FP64;
  // set_dimension
  int nspins = 0, nkpts = 0, nstates = 0, nbasis = 0, natoms = 0;
  // set_wg_ekb_efermi: [nkpts][nstates]
  std::vector<double> wg, ekb;
  double efermi = 0.0;
  bool have_bands = false;
  // set_ao_basis_wfc: c_{i n}(k) at [k][i][n] (complex interleaved)
  std::vector<double> wfc;
  std::vector<char> have_wfc;
  // lattice (rows) and reciprocal vectors (rows), k mesh and k vectors (Cartesian)
  double lat[9] = {0}, G[9] = {0};
  bool have_lat = false;
  int mesh[3] = {0, 0, 0};
  std::vector<double> kvec;
  // irreducible k points: indices into the k list and weights
  std::vector<int> irk;
  std::vector<double> wirk;
  // LRI blocks keyed by (I, J, R)
  std::map<std::tuple<int, int, int, int, int>, AuxBlock> aux;
  // Coulomb matrices per irreducible q point (complex [naux][naux]), filled blockwise
  std::map<int, std::vector<double>> vq;
  std::map<int, std::vector<char>> vq_set;
  // time / frequency grids
  int ngrid = 0;
  std::vector<double> tau, womega, gamma_cos;
};

namespace {

int fail(rpa_session *s, int code, const std::string &m) {
  s->err = m;
  return code;
}

// Per-atom NAO and ABF counts as the LRI blocks give them (the ABF index of a block sits on I).
bool atom_sizes(rpa_session *s, std::vector<int> &nao, std::vector<int> &naux, std::string &why) {
  nao.assign(s->natoms, 0);
  naux.assign(s->natoms, 0);
  for (auto &kv : s->aux) {
    const AuxBlock &b = kv.second;
    auto put = [&](std::vector<int> &v, int a, int n) {
      if (v[a] == 0) v[a] = n;
      return v[a] == n;
    };
    if (!put(nao, b.I, b.ni) || !put(nao, b.J, b.nj) || !put(naux, b.I, b.na)) {
      why = "inconsistent basis sizes for atom " + std::to_string(b.I) + " or " + std::to_string(b.J);
      return false;
    }
  }
  for (int a = 0; a < s->natoms; ++a)
    if (nao[a] <= 0 || naux[a] <= 0) {
      why = "atom " + std::to_string(a) + " has no LRI block of its own";
      return false;
    }
  return true;
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc(&p, n > 0 ? n : 1); }
  template <typename T> T *as() const { return (T *)p; }
};

}  // namespace

extern "C" {

int rpa_session_create(rpa_ctx *ctx, rpa_session **out) {
  if (!ctx || !out) return RPA_ERR_ARG;
  rpa_session *s = new rpa_session();
  s->ctx = ctx;
  *out = s;
  return RPA_OK;
}

int rpa_session_destroy(rpa_session *s) {
  if (!s) return RPA_ERR_ARG;
  delete s;
  return RPA_OK;
}

const char *rpa_session_last_error(const rpa_session *s) { return s ? s->err.c_str() : "null session"; }

int rpa_session_set_precision(rpa_session *s, int precision) {
  if (!s) return RPA_ERR_ARG;
  if (precision != RPA_FP64 && precision != RPA_FP32 && precision != RPA_BF16X3)
    return fail(s, RPA_ERR_ARG, "unknown precision");
  s->precision = precision;
  return RPA_OK;
}

int rpa_set_dimension(rpa_session *s, int nspins, int nkpts, int nstates, int nbasis, int natoms) {
  if (!s) return RPA_ERR_ARG;
  if (nspins <= 0 || nkpts <= 0 || nstates <= 0 || nbasis <= 0 || natoms <= 0)
    return fail(s, RPA_ERR_ARG, "dimensions must be positive");
  if (nspins != 1) return fail(s, RPA_ERR_UNSUPPORTED, "closed shells only (nspins = 1)");
  if (nstates > nbasis) return fail(s, RPA_ERR_SHAPE, "more states than basis functions");
  s->nspins = nspins;
  s->nkpts = nkpts;
  s->nstates = nstates;
  s->nbasis = nbasis;
  s->natoms = natoms;
  s->wfc.assign((size_t)nkpts * nbasis * nstates * 2, 0.0);
  s->have_wfc.assign(nkpts, 0);
  s->have_bands = false;
  return RPA_OK;
}

int rpa_set_wg_ekb_efermi(rpa_session *s, int nspins, int nkpts, int nstates, const double *wg, const double *ekb,
                          double efermi) {
  if (!s) return RPA_ERR_ARG;
  if (!wg || !ekb) return fail(s, RPA_ERR_ARG, "null argument");
  if (nspins != s->nspins || nkpts != s->nkpts || nstates != s->nstates)
    return fail(s, RPA_ERR_SHAPE, "dimensions differ from set_dimension");
  s->wg.assign(wg, wg + (size_t)nkpts * nstates);
  s->ekb.assign(ekb, ekb + (size_t)nkpts * nstates);
  s->efermi = efermi;
  s->have_bands = true;
  return RPA_OK;
}

int rpa_set_ao_basis_wfc(rpa_session *s, int ispin, int ik, const double *wfc_real, const double *wfc_imag) {
  if (!s) return RPA_ERR_ARG;
  if (!wfc_real || !wfc_imag) return fail(s, RPA_ERR_ARG, "null argument");
  if (s->nkpts == 0) return fail(s, RPA_ERR_SHAPE, "set_dimension first");
  if (ispin != 0 || ik < 0 || ik >= s->nkpts) return fail(s, RPA_ERR_ARG, "spin or k index out of range");
  // input [n][i] (band-major); stored as c_{i n}(k) at [k][i][n]
  const int nb = s->nbasis, ns = s->nstates;
  double *dst = s->wfc.data() + (size_t)ik * nb * ns * 2;
  for (int n = 0; n < ns; ++n)
    for (int i = 0; i < nb; ++i) {
      dst[((size_t)i * ns + n) * 2] = wfc_real[(size_t)n * nb + i];
      dst[((size_t)i * ns + n) * 2 + 1] = wfc_imag[(size_t)n * nb + i];
    }
  s->have_wfc[ik] = 1;
  return RPA_OK;
}

int rpa_set_latvec_and_G(rpa_session *s, const double lat_mat[9], const double G_mat[9]) {
  if (!s) return RPA_ERR_ARG;
  if (!lat_mat || !G_mat) return fail(s, RPA_ERR_ARG, "null argument");
  std::memcpy(s->lat, lat_mat, sizeof s->lat);
  std::memcpy(s->G, G_mat, sizeof s->G);
  s->have_lat = true;
  return RPA_OK;
}

int rpa_set_kgrids_kvec_tot(rpa_session *s, int nk1, int nk2, int nk3, const double *kvecs) {
  if (!s) return RPA_ERR_ARG;
  if (!kvecs) return fail(s, RPA_ERR_ARG, "null argument");
  if (nk1 <= 0 || nk2 <= 0 || nk3 <= 0) return fail(s, RPA_ERR_ARG, "mesh must be positive");
  if (s->nkpts == 0 || nk1 * nk2 * nk3 != s->nkpts)
    return fail(s, RPA_ERR_SHAPE, "mesh size differs from the k-point count of set_dimension");
  s->mesh[0] = nk1;
  s->mesh[1] = nk2;
  s->mesh[2] = nk3;
  s->kvec.assign(kvecs, kvecs + 3 * (size_t)s->nkpts);
  return RPA_OK;
}

int rpa_set_ibz2bz_index_and_weight(rpa_session *s, int nk_irk, const int *ibz2bz_index, const double *wk_irk) {
  if (!s) return RPA_ERR_ARG;
  if (nk_irk <= 0 || !ibz2bz_index || !wk_irk) return fail(s, RPA_ERR_ARG, "bad irreducible k list");
  double sum = 0.0;
  for (int i = 0; i < nk_irk; ++i) {
    if (ibz2bz_index[i] < 0 || ibz2bz_index[i] >= s->nkpts || !(wk_irk[i] > 0.0))
      return fail(s, RPA_ERR_ARG, "irreducible k index or weight out of range");
    sum += wk_irk[i];
  }
  s->irk.assign(ibz2bz_index, ibz2bz_index + nk_irk);
  s->wirk.assign(wk_irk, wk_irk + nk_irk);
  for (double &w : s->wirk) w /= sum;
  s->vq.clear();
  s->vq_set.clear();
  return RPA_OK;
}

int rpa_set_ao_basis_aux(rpa_session *s, int I, int J, int nbasis_i, int nbasis_j, int naux_mu, const int *R,
                         const double *Cs_in, int insert_index_only) {
  if (!s) return RPA_ERR_ARG;
  if (!R || (!insert_index_only && !Cs_in)) return fail(s, RPA_ERR_ARG, "null argument");
  if (s->natoms == 0) return fail(s, RPA_ERR_SHAPE, "set_dimension first");
  if (I < 0 || I >= s->natoms || J < 0 || J >= s->natoms || nbasis_i <= 0 || nbasis_j <= 0 || naux_mu <= 0)
    return fail(s, RPA_ERR_ARG, "atom index or block size out of range");
  AuxBlock &b = s->aux[std::make_tuple(I, J, R[0], R[1], R[2])];
  b.I = I;
  b.J = J;
  b.ni = nbasis_i;
  b.nj = nbasis_j;
  b.na = naux_mu;
  for (int d = 0; d < 3; ++d) b.R[d] = R[d];
  const size_t n = (size_t)naux_mu * nbasis_i * nbasis_j;
  if (insert_index_only)
    b.C.assign(n, 0.0);
  else
    b.C.assign(Cs_in, Cs_in + n);
  return RPA_OK;
}

// Coulomb matrix of irreducible q point ik (index into the irreducible list, or into the k list
// when none was given): its block [mu_begin, mu_end) x [nu_begin, nu_end) of the whole
// max_naux x max_naux matrix, real and imaginary parts row-major.
int rpa_set_aux_bare_coulomb_k_2D_block(rpa_session *s, int ik, int max_naux, int mu_begin, int mu_end, int nu_begin,
                                        int nu_end, const double *Vq_real_in, const double *Vq_imag_in) {
  if (!s) return RPA_ERR_ARG;
  if (!Vq_real_in || !Vq_imag_in) return fail(s, RPA_ERR_ARG, "null argument");
  const int nq = s->irk.empty() ? s->nkpts : (int)s->irk.size();
  if (ik < 0 || ik >= nq) return fail(s, RPA_ERR_ARG, "q index out of range");
  if (max_naux <= 0 || mu_begin < 0 || nu_begin < 0 || mu_end > max_naux || nu_end > max_naux ||
      mu_begin > mu_end || nu_begin > nu_end)
    return fail(s, RPA_ERR_ARG, "block out of range");
  std::vector<double> &v = s->vq[ik];
  std::vector<char> &set = s->vq_set[ik];
  if (v.empty()) {
    v.assign((size_t)max_naux * max_naux * 2, 0.0);
    set.assign((size_t)max_naux * max_naux, 0);
  } else if (v.size() != (size_t)max_naux * max_naux * 2) {
    return fail(s, RPA_ERR_SHAPE, "max_naux differs from an earlier block of this q point");
  }
  const int w = nu_end - nu_begin;
  for (int m = mu_begin; m < mu_end; ++m)
    for (int n = nu_begin; n < nu_end; ++n) {
      const size_t src = (size_t)(m - mu_begin) * w + (n - nu_begin), dst = (size_t)m * max_naux + n;
      v[2 * dst] = Vq_real_in[src];
      v[2 * dst + 1] = Vq_imag_in[src];
      set[dst] = 1;
    }
  return RPA_OK;
}

int rpa_set_aux_bare_coulomb_k_atom_pair(rpa_session *s, int ik, int I, int J, int naux_mu, int naux_nu,
                                         const double *Vq_real_in, const double *Vq_imag_in) {
  if (!s) return RPA_ERR_ARG;
  std::vector<int> nao, naux;
  std::string why;
  if (!atom_sizes(s, nao, naux, why)) return fail(s, RPA_ERR_SHAPE, "set the LRI blocks first: " + why);
  if (I < 0 || I >= s->natoms || J < 0 || J >= s->natoms) return fail(s, RPA_ERR_ARG, "atom index out of range");
  if (naux_mu != naux[I] || naux_nu != naux[J]) return fail(s, RPA_ERR_SHAPE, "ABF counts differ from the LRI blocks");
  int off_i = 0, off_j = 0, tot = 0;
  for (int a = 0; a < s->natoms; ++a) {
    if (a == I) off_i = tot;
    if (a == J) off_j = tot;
    tot += naux[a];
  }
  return rpa_set_aux_bare_coulomb_k_2D_block(s, ik, tot, off_i, off_i + naux_mu, off_j, off_j + naux_nu, Vq_real_in,
                                             Vq_imag_in);
}

int rpa_set_time_freq_grids(rpa_session *s, int ngrid, const double *tau, const double *omega_weights,
                            const double *gamma_cos) {
  if (!s) return RPA_ERR_ARG;
  if (ngrid <= 0 || !tau || !omega_weights || !gamma_cos) return fail(s, RPA_ERR_ARG, "bad grids");
  s->ngrid = ngrid;
  s->tau.assign(tau, tau + ngrid);
  s->womega.assign(omega_weights, omega_weights + ngrid);
  s->gamma_cos.assign(gamma_cos, gamma_cos + (size_t)ngrid * ngrid);
  return RPA_OK;
}

int rpa_get_rpa_correlation_energy(rpa_session *s, double *rpa_corr, double *rpa_corr_irk_contrib) {
  if (!s) return RPA_ERR_ARG;
  if (!rpa_corr) return fail(s, RPA_ERR_ARG, "null argument");
  rpa_ctx *ctx = s->ctx;
  // ---- completeness and shapes of the inputs
  if (s->natoms == 0) return fail(s, RPA_ERR_SHAPE, "set_dimension missing");
  if (!s->have_bands) return fail(s, RPA_ERR_SHAPE, "set_wg_ekb_efermi missing");
  for (int k = 0; k < s->nkpts; ++k)
    if (!s->have_wfc[k]) return fail(s, RPA_ERR_SHAPE, "eigenvectors missing at k index " + std::to_string(k));
  if (!s->have_lat || s->kvec.empty()) return fail(s, RPA_ERR_SHAPE, "lattice or k grid missing");
  if (s->ngrid == 0) return fail(s, RPA_ERR_SHAPE, "time / frequency grids missing");
  std::vector<int> nao, naux;
  std::string why;
  if (!atom_sizes(s, nao, naux, why)) return fail(s, RPA_ERR_SHAPE, why);
  int nb = 0, N = 0;
  for (int a = 0; a < s->natoms; ++a) {
    nb += nao[a];
    N += naux[a];
  }
  if (nb != s->nbasis) return fail(s, RPA_ERR_SHAPE, "the LRI blocks' NAO counts do not add up to nbasis");
  // occupied bands: weight above half the largest, the same count at every k (an insulator)
  double wmax = 0.0;
  for (double w : s->wg) wmax = std::max(wmax, std::fabs(w));
  int nocc = -1;
  for (int k = 0; k < s->nkpts; ++k) {
    int n = 0;
    for (int b = 0; b < s->nstates; ++b) n += std::fabs(s->wg[(size_t)k * s->nstates + b]) > 0.5 * wmax;
    for (int b = 0; b < s->nstates; ++b)
      if ((std::fabs(s->wg[(size_t)k * s->nstates + b]) > 0.5 * wmax) != (b < n))
        return fail(s, RPA_ERR_UNSUPPORTED, "occupied bands must come first at every k");
    if (nocc >= 0 && n != nocc) return fail(s, RPA_ERR_UNSUPPORTED, "the occupied-band count must not depend on k");
    nocc = n;
  }
  // fractional k (and q) coordinates: k . a_d / (2 pi)
  std::vector<double> kfrac((size_t)s->nkpts * 3);
  for (int k = 0; k < s->nkpts; ++k)
    for (int d = 0; d < 3; ++d) {
      double x = 0.0;
      for (int c = 0; c < 3; ++c) x += s->kvec[3 * k + c] * s->lat[3 * d + c];
      kfrac[3 * k + d] = x / (2.0 * M_PI);
    }
  const bool ibz = !s->irk.empty();
  const int nq = ibz ? (int)s->irk.size() : s->nkpts;
  std::vector<double> qfrac((size_t)nq * 3), wq(nq);
  for (int i = 0; i < nq; ++i) {
    const int k = ibz ? s->irk[i] : i;
    for (int d = 0; d < 3; ++d) qfrac[3 * i + d] = kfrac[3 * k + d];
    wq[i] = ibz ? s->wirk[i] : 1.0 / nq;
  }
  for (int i = 0; i < nq; ++i) {
    auto it = s->vq_set.find(i);
    if (it == s->vq_set.end() || s->vq[i].size() != (size_t)N * N * 2 ||
        std::find(it->second.begin(), it->second.end(), 0) != it->second.end())
      return fail(s, RPA_ERR_SHAPE, "Coulomb matrix incomplete at q index " + std::to_string(i));
  }
  // LRI block list in insertion-independent order and the coefficients side by side
  const int nblk = (int)s->aux.size();
  std::vector<int> bI, bK, bR;
  std::vector<long long> boff;
  std::vector<double> Ch;
  for (auto &kv : s->aux) {
    const AuxBlock &b = kv.second;
    bI.push_back(b.I);
    bK.push_back(b.J);
    for (int d = 0; d < 3; ++d) bR.push_back(b.R[d]);
    boff.push_back((long long)Ch.size());
    Ch.insert(Ch.end(), b.C.begin(), b.C.end());
  }
  // ---- plan and device buffers
  const int nt = s->ngrid, nR = s->mesh[0] * s->mesh[1] * s->mesh[2];
  rpa_cell cell{s->natoms, nao.data(), naux.data(), {s->mesh[0], s->mesh[1], s->mesh[2]}};
  rpa_lri_blocks blocks{nblk, bI.data(), bK.data(), bR.data(), boff.data()};
  rpa_plan *plan = nullptr;
  size_t wsb = 0;
  int rc = rpa_plan_create(ctx, &cell, &blocks, nt, s->precision, &wsb, &plan);
  if (rc != RPA_OK) return fail(s, rc, std::string("plan: ") + rpa_last_error(ctx));
  struct PlanGuard {
    rpa_plan *p;
    ~PlanGuard() { rpa_plan_destroy(p); }
  } guard{plan};
  const size_t n2 = (size_t)N * N;
  const size_t gsz = (size_t)nt * nR * nb * nb;
  const size_t big = std::max((size_t)nt * nR * n2, (size_t)2 * nt * nq * n2);   // chi(tau), later chi(q)
  const size_t gws = rpa_green_workspace_size(s->nkpts, nb, nocc);
  const size_t ews = rpa_ec_workspace_size(N, nq, nt);
  DevBuf dC, dEps, dWfc, dG, dGws, dChi, dChiW, dV, dWs, dEws;
  hipError_t he = hipSuccess;
  if ((he = dC.alloc(Ch.size() * 8)) != hipSuccess || (he = dEps.alloc(s->ekb.size() * 8)) != hipSuccess ||
      (he = dWfc.alloc(s->wfc.size() * 8)) != hipSuccess || (he = dG.alloc(2 * gsz * 8)) != hipSuccess ||
      (he = dGws.alloc(gws)) != hipSuccess || (he = dChi.alloc(big * 8)) != hipSuccess ||
      (he = dChiW.alloc((size_t)nt * nR * n2 * 8)) != hipSuccess || (he = dV.alloc((size_t)nq * n2 * 16)) != hipSuccess ||
      (he = dWs.alloc(wsb)) != hipSuccess || (he = dEws.alloc(ews)) != hipSuccess)
    return fail(s, RPA_ERR_HIP, std::string("device buffers: ") + hipGetErrorString(he));
  std::vector<double> vq_all((size_t)nq * n2 * 2);
  for (int i = 0; i < nq; ++i) std::copy(s->vq[i].begin(), s->vq[i].end(), vq_all.begin() + (size_t)i * n2 * 2);
  if ((he = hipMemcpy(dC.p, Ch.data(), Ch.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(dEps.p, s->ekb.data(), s->ekb.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(dWfc.p, s->wfc.data(), s->wfc.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(dV.p, vq_all.data(), vq_all.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(s, RPA_ERR_HIP, std::string("upload: ") + hipGetErrorString(he));
  double *Go = dG.as<double>(), *Gu = Go + gsz;
  // ---- the path: G(R, tau) from the eigenpairs, chi0(R, tau), transforms, E_c
  rc = build_green_tau(ctx, s->nkpts, nb, nocc, s->efermi, nt, s->tau.data(), s->mesh, kfrac.data(), dEps.as<double>(),
                       dWfc.as<double>(), dGws.p, gws, Go, Gu);
  if (rc == RPA_OK)
    rc = build_chi0_tau(plan, 2.0, Go, Gu, dC.as<double>(), dWs.p, wsb, dChi.as<double>());   // closed shell
  if (rc == RPA_OK)
    rc = chi0_tau_to_omega(ctx, nt, nt, (size_t)nR * n2, s->gamma_cos.data(), dChi.as<double>(), dChiW.as<double>());
  if (rc == RPA_OK)
    rc = chi0_R_to_q(ctx, s->mesh, nt, n2, nq, qfrac.data(), dChiW.as<double>(), dChi.as<double>());
  std::vector<double> ecq(nq);
  double ec = 0.0;
  if (rc == RPA_OK)
    rc = rpa_correlation_energy(ctx, N, nq, nt, s->womega.data(), dChi.as<double>(), dV.as<double>(), dEws.p, ews, &ec,
                                ecq.data());
  if (rc != RPA_OK) return fail(s, rc, rpa_last_error(ctx));
  // per-q terms come divided by nq; irreducible points carry their weights instead
  if (!ibz) {
    if (rpa_corr_irk_contrib) std::copy(ecq.begin(), ecq.end(), rpa_corr_irk_contrib);
    *rpa_corr = ec;
    return RPA_OK;
  }
  double tot = 0.0;
  for (int i = 0; i < nq; ++i) {
    const double c = ecq[i] * nq * wq[i];
    if (rpa_corr_irk_contrib) rpa_corr_irk_contrib[i] = c;
    tot += c;
  }
  *rpa_corr = tot;
  return RPA_OK;
}

}  // extern "C"
