// C ABI of the chi0 -> E_c library (declared in include/rpa_mi355x.h): contexts,
// plans (neighbour tables and work lists of Algorithm 1) and the four compute calls.
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rpa_mi355x.h"
#include "chi0_kernels.h"
#include "ec_kernels.h"
#include "green_kernels.h"

hipError_t launch_cos_transform(const double *W_dev, int ntau, int nomega, size_t n, const double *x, double *y,
                                hipStream_t s);
hipError_t launch_r2q(const double *ph_dev, int nR, int nq, int nbatch, size_t m, const double *x, double *y,
                      hipStream_t s);

struct rpa_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  double *params = nullptr;        // small device buffer for per-call weights and phases
  size_t params_bytes = 0;
  std::string err;
  // opt-in kernel timing
  bool profile = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, int>> totals;
  // autotuner choices by plan shape class and device architecture
  std::map<std::string, rpa_tuning> tune_cache;
  // device address of the no-allocation scratch array on this context's device
  void *scratch = nullptr;
};

namespace {

constexpr size_t kParamsBytes = 1 << 20;

int fail(rpa_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((ctx), RPA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Plan tables live in device memory.  The host-only build of the table code (RPA_HOST_TABLE_TEST,
// compiled by the sanitizer test with address and undefined-behaviour checks on the host code)
// keeps them in host memory instead and launches no kernel.
#ifdef RPA_HOST_TABLE_TEST
hipError_t table_alloc(int, void **p, size_t n) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t table_upload(void *dst, const void *src, size_t n) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
void table_free(int, void *p) { std::free(p); }
#else
hipError_t table_alloc(int device, void **p, size_t n) {
  hipError_t e = hipSetDevice(device);
  return e == hipSuccess ? hipMalloc(p, n) : e;
}
hipError_t table_upload(void *dst, const void *src, size_t n) {
  return hipMemcpy(dst, src, n, hipMemcpyHostToDevice);
}
void table_free(int device, void *p) {
  // the tables may still be read by queued kernels of the plan
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  (void)hipFree(p);
}
#endif

hipError_t scratch_setup(int device, void **out);   // device scratch of the no-allocation entry point

// Records HIP events around the enclosed launches when profiling is on.
struct Timed {
  rpa_ctx *ctx;
  const char *name;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(rpa_ctx *c, const char *n) : ctx(c), name(n) {
    if (ctx->profile && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      hipEventRecord(a, ctx->stream);
  }
  ~Timed() {
    if (a && b) {
      hipEventRecord(b, ctx->stream);
      ctx->pending.push_back({name, a, b});
    }
  }
};

// Order of a work list of n entries in which workgroup b (dealt to XCD b % 8) runs entry
// perm[b]: XCD x gets the contiguous range [x q + min(x, r), ...) of the plain order, q = n / 8,
// r = n % 8, so that the entries one XCD runs are neighbours in the plain order.
std::vector<int> xcd_grouped_order(int n) {
  std::vector<int> perm(n);
  const int q = n / 8, r = n % 8;
  for (int b = 0; b < n; ++b) {
    const int x = b % 8;
    perm[b] = x * q + std::min(x, r) + b / 8;
  }
  return perm;
}

int drain_profile(rpa_ctx *ctx) {
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return RPA_ERR_HIP;
    auto &t = ctx->totals[p.name];
    t.first += ms;
    t.second += 1;
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  ctx->pending.clear();
  return RPA_OK;
}

}  // namespace

struct PlanGroup {
  int mt, js, hc, start, count;
};

struct rpa_plan {
  rpa_ctx *ctx = nullptr;      // must outlive the plan
  int device = 0;
  int natoms = 0, nb = 0, nauxtot = 0, nR = 0, ntau = 0, prec = 0, nblk = 0;
  int mesh[3] = {1, 1, 1};
  Bvk bvk{1, 1, 1};
  std::vector<int> nao, naux, ao_off, aux_off, atom_of_ao;
  std::vector<long long> in_off, out_off;      // caller block offsets, packed offsets
  std::vector<long long> cb_off;                // split-BF16 packed offsets (bf16 elements)
  long long cb_elems = 0;
  std::vector<int> blk_a, blk_ni, blk_nk, blk_stride;
  std::vector<int> cp_stride;                   // per atom: packed row length, nao*naux rounded up to 8
  int nbp = 0;                                  // nb rounded up to 8
  long long cp_elems = 0, maxblk = 0;
  std::vector<int> nbr_start, nbr_K, nbr_R1, nbr_run_end;
  std::vector<long long> nbr_cp, nbr_cb;
  std::vector<int> nslices;                     // per atom U: sum of n_K over its neighbours
  std::vector<int> rows_start;
  std::vector<int4> row_info;
  std::vector<long long> noff, noffs;
  long long n_elems = 0;                        // N buffer elements per tau
  long long ns_elems = 0;                       // split-BF16 N elements per tau (BF16X3 plans)
  std::vector<int> tileV, tileM, tileN;
  std::vector<int> tile2V, tile2M, tile2N;     // tiles of 256 rows (split-BF16 N stage)
  std::vector<int> itemU, itemV, itemR;
  std::vector<PlanGroup> groups;
  double alg_flops = 0, exec_flops = 0;
  double stage_alg[2] = {0, 0}, stage_exec[2] = {0, 0};
  // device tables (one allocation owned by the plan)
  void *dtab = nullptr;
  Chi0Tables tb{};
  NTiles tiles{};
  PairItems items{};
  PackTables pack{};
  const int *dgsrc = nullptr;
  // XCD-grouped orders of the same tiles and items (items permuted within each group)
  NTiles tiles_x{};
  NTiles tiles2{}, tiles2_x{};
  PairItems items_x{};
  rpa_tuning tune{0, 16, 0, 0, 0.0, 0.0, 0, 128};
  std::string shape_key;                        // autotuner cache key (without the architecture)
  // split-BF16 N stage (BF16X3 plans whose hi and lo parts of transposed G and C each fit a
  // 32-bit buffer view; other BF16X3 plans run the FP32 N stage)
  bool nbf16 = false;
  int nbq = 0;                                  // GT columns: sum of nao rounded up to 8
  std::vector<int> aopad_off, gsrc;             // per atom GT column offset; GT column -> NAO or -1
  std::vector<long long> ctn_off;               // per block CtN offset (bf16 elements)
  long long ctn_elems = 0;
  std::vector<int> ngrp_start;
  std::vector<int4> ngrp;
  std::vector<long long> ngrp_off;
  unsigned gt_bytes = 0, ct_bytes = 0;          // one part (hi or lo)
  // workspace layout (bytes); the per-tau parts (padded G, N, transposed G, G-scale exponents)
  // are held for `slots` tau points at once, g_slot, n_slot, gt_slot bytes apart
  size_t ws_cp = 0, ws_cb = 0, ws_g = 0, ws_n = 0, ws_sc = 0, ws_gt = 0, ws_ct = 0, ws_total = 0;
  size_t g_slot = 0, n_slot = 0, gt_slot = 0, ns_slot = 0, ws_ns = 0;
  int slots = 1;                                // tau points per N-stage / fused launch
  // single fused launch of the split-BF16 path: per plan item its class code and the items in
  // order of decreasing work
  std::vector<int> item_cls, item_order, half_order;   // half_order: 2 item + half (4-wave units)
  const int *d_item_cls = nullptr, *d_item_order = nullptr, *d_half_order = nullptr;
  // Green's-function screening (off while theta == 0): a plan-owned device buffer with the
  // bounds of one tau (gb, gn, gc) and the per-item statistics of every tau of the last build
  double theta = 0.0;
  void *dscr = nullptr;
  double *scr_gb = nullptr, *scr_gn = nullptr, *scr_gc = nullptr;
  int *scr_stats = nullptr;                     // [ntau][items][3]
  bool scr_valid = false;                       // statistics of a complete build are present

  PairItems group_items(const PlanGroup &g, int order = 0) const {
    const PairItems &it = order ? items_x : items;
    return PairItems{it.U + g.start, it.V + g.start, it.R + g.start, g.count};
  }
  const NTiles &ntiles(int order, int bm = 128) const {
    return bm == 256 ? (order ? tiles2_x : tiles2) : (order ? tiles_x : tiles);
  }
};

// ---- correlation energy ----
namespace {
struct EcLayout {
  size_t L, T, B, W, trB, f, flags, ecq, w, realq, realv, rboth, rpair, counts, total;
  int cw;
};
// L: Cholesky factors of v(q) for every q; T, B: cw (q, omega) matrices at a time.  At a q
// where chi and v are both real the slots hold real row-major matrices: L_q in the first n^2
// doubles of its slot, Re chi(q, omega) and then T in the two halves of a T slot, B in the
// first half of a B slot.
EcLayout ec_layout(int n, int nq, int nomega, int cw) {
  EcLayout l{};
  const size_t mat = (size_t)n * n * 16;
  size_t o = 0;
  l.L = o;
  o = align_up(o + mat * nq);
  l.T = o;
  o = align_up(o + mat * cw);
  l.B = o;
  o = align_up(o + mat * cw);
  l.W = o;
  o = align_up(o + (size_t)std::max(cw, nq) * kCholBlock * kCholBlock * 16);
  l.trB = o;
  o = align_up(o + (size_t)nq * nomega * 8);
  l.f = o;
  o = align_up(o + (size_t)nq * nomega * 8);
  l.flags = o;
  o = align_up(o + (size_t)(nq + nq * nomega) * 4);
  l.ecq = o;
  o = align_up(o + (size_t)(nq + 1) * 8);
  l.w = o;
  o = align_up(o + (size_t)nomega * 8);
  l.realq = o;
  o = align_up(o + (size_t)nq * 4);
  l.realv = o;
  o = align_up(o + (size_t)nq * 4);
  l.rboth = o;
  o = align_up(o + (size_t)nq * 4);
  l.rpair = o;
  o = align_up(o + (size_t)nq * nomega * 4);
  l.counts = o;
  o = align_up(o + 2 * 4);
  l.total = o;
  l.cw = cw;
  return l;
}
// (q, omega) pairs per batch for the default workspace: all of them, up to 64 GiB of the two
// per-pair matrices T and B (24 pairs of order 7440 take 42 GB).  Each batch runs its own
// sequence of n / 32 Cholesky panel steps, whose diagonal-block kernel costs about the same for
// one matrix as for many, so fewer and larger batches finish sooner.
int ec_default_batch(int n, int nq, int nomega) {
  const size_t mat = (size_t)n * n * 16;
  const size_t cap = std::max<size_t>(1, ((size_t)64 << 30) / (2 * mat));
  return (int)std::min<size_t>((size_t)nq * nomega, cap);
}
}  // namespace

// T: precision of G, N and the N stage; bf16: split-BF16 fused kernel (T = float).  G is rescaled
// per tau by a power of two in the FP32 and BF16X3 paths.
namespace {
// Largest (q, omega) batch whose layout fits the workspace; false if even one matrix does not.
bool ec_fit_layout(int n, int nq, int nomega, size_t workspace_bytes, EcLayout &out) {
  const int total = nq * nomega;
  int cw = std::min(total, std::max(1, ec_default_batch(n, nq, nomega)));
  while (cw > 1 && ec_layout(n, nq, nomega, cw).total > workspace_bytes) cw = (cw + 1) / 2;
  while (cw < total && ec_layout(n, nq, nomega, cw + 1).total <= workspace_bytes) ++cw;
  out = ec_layout(n, nq, nomega, cw);
  return out.total <= workspace_bytes;
}

// Status flags written by the energy stage: [nq] for the Cholesky of v(q), then
// [nq][nomega] for 1 - L^H chi L (1: not positive definite, 2: non-finite log-determinant).
int ec_check_flags(rpa_ctx *ctx, const int *hflags, int nq, int nomega, const std::string &where) {
  for (int q = 0; q < nq; ++q) {
    if (hflags[q] == 2)
      return fail(ctx, RPA_ERR_NONFINITE, where + "NaN or Inf in v(q) at q index " + std::to_string(q));
    if (hflags[q])
      return fail(ctx, RPA_ERR_NOT_HPD, where + "v(q) is not Hermitian positive definite at q index " + std::to_string(q));
  }
  for (int q = 0; q < nq; ++q)
    for (int k = 0; k < nomega; ++k) {
      const int fl = hflags[nq + q * nomega + k];
      if (fl == 1)
        return fail(ctx, RPA_ERR_NOT_HPD, where + "1 - L^H chi L is not positive definite at q index " +
                                              std::to_string(q) + ", omega index " + std::to_string(k));
      if (fl == 2)
        return fail(ctx, RPA_ERR_NONFINITE, where + "non-finite log-determinant at q index " + std::to_string(q) +
                                                ", omega index " + std::to_string(k));
    }
  return RPA_OK;
}

// First part of the energy stage: status flags cleared, and the kinds of the q points found on
// the device (realq: chi real; realv: v real; rboth: both, the real layout; rpair: rboth per
// (q, omega) pair; counts: {q points with the real layout, the others}).
int ec_flags_enqueue(rpa_ctx *ctx, hipStream_t s, int n, int nq, int nomega, const double *chi0_q,
                     const double *v_q, char *ws, const EcLayout &l) {
  int *flags = (int *)(ws + l.flags), *realq = (int *)(ws + l.realq), *realv = (int *)(ws + l.realv),
      *rboth = (int *)(ws + l.rboth), *rpair = (int *)(ws + l.rpair), *counts = (int *)(ws + l.counts);
  HIP_TRY(ctx, launch_fill_int(flags, (size_t)(nq + nq * nomega), 0, s));
  // q points whose chi(q, i omega) is real at every omega (time-reversal invariant q, where the
  // phases of R -> q are +1 or -1): T = chi L there takes two real products per complex one;
  // where v(q) is real too, every step of that q runs on real matrices
  HIP_TRY(ctx, launch_real_flags(chi0_q, n, nq, nomega, realq, s));
  HIP_TRY(ctx, launch_real_flags(v_q, n, nq, 1, realv, s));
  HIP_TRY(ctx, launch_both_real(realq, realv, nq, nomega, rboth, rpair, counts, s));
  return RPA_OK;
}

// The rest of the stage.  kinds: bit 0 if complex-layout q points may be present, bit 1 if
// real-layout ones may; the kernels of an absent kind are not launched (the kernels of a present
// kind skip the matrices of the other one).
int ec_main_enqueue(rpa_ctx *ctx, hipStream_t s, int n, int nq, int nomega, const double *womega_dev,
                    const double *chi0_q, const double *v_q, char *ws, const EcLayout &l, int kinds) {
  const int total = nq * nomega, cw = l.cw;
  double *L = (double *)(ws + l.L), *T = (double *)(ws + l.T), *B = (double *)(ws + l.B),
         *W = (double *)(ws + l.W), *trB = (double *)(ws + l.trB), *f = (double *)(ws + l.f),
         *ecq = (double *)(ws + l.ecq);
  int *flags = (int *)(ws + l.flags), *realq = (int *)(ws + l.realq), *rboth = (int *)(ws + l.rboth),
      *rpair = (int *)(ws + l.rpair);
  const bool cplx = kinds & 1, rl = kinds & 2;
  const size_t mat = (size_t)n * n * 2;   // doubles per complex matrix
  const size_t n2 = (size_t)n * n;
  // v(q) = L_q L_q^H for every q at once
  if (cplx) HIP_TRY(ctx, launch_copy_words(L, v_q, nq * mat * 2, s));
  if (rl) HIP_TRY(ctx, launch_pack_real(v_q, (long long)mat, 0, 0, 1, nq, L, mat, n2, rboth, s));
  HIP_TRY(ctx, launch_cholesky(L, mat, n, nq, W, flags, 0, rboth, s, kinds));
  HIP_TRY(ctx, launch_zero_upper(L, mat, n, nq, rboth, s));
  // (q, omega) pairs g = q * nomega + omega in batches of cw
  for (int b0 = 0; b0 < total; b0 += cw) {
    const int nb = std::min(cw, total - b0);
    // T = chi(q, omega) L_q   (L_q lower triangular: k >= first column of the tile)
    ZgemmArgs g{};
    g.M = g.N = g.K = n;
    g.A = chi0_q;
    g.lda = n;
    g.outerA = (long long)mat;                 // q
    g.innerA = (long long)nq * mat;            // omega
    g.opA = 0;
    g.B = L;
    g.ldb = n;
    g.outerB = (long long)mat;
    g.opB = 0;
    g.C = T;
    g.ldc = n;
    g.strideC = (long long)mat;
    g.boff = b0;
    g.binner = nomega;
    g.alpha = 1.0;
    g.kmode = 1;
    g.realA = realq;
    g.skip = rboth;
    if (cplx) HIP_TRY(ctx, launch_zgemm(g, nb, s));
    // the real pairs: Re chi into the first half of the T slot, T = chi L into the second
    if (rl)
      HIP_TRY(ctx, launch_pack_real(chi0_q, (long long)mat, (long long)nq * mat, b0, nomega, nb, T, mat, n2, rboth, s));
    DgemmArgs gr{};
    gr.M = gr.N = gr.K = n;
    gr.A = T;
    gr.lda = n;
    gr.strideA = (long long)mat;
    gr.B = L;
    gr.ldb = n;
    gr.outerB = (long long)mat;
    gr.C = T + n2;
    gr.ldc = n;
    gr.strideC = (long long)mat;
    gr.boff = b0;
    gr.binner = nomega;
    gr.alpha = 1.0;
    gr.kmode = 1;
    gr.sel = rboth;
    if (rl) HIP_TRY(ctx, launch_dgemm(gr, nb, s));
    // B = L_q^H T, lower triangle (L^H upper triangular: k >= first row of the tile)
    ZgemmArgs h{};
    h.M = h.N = h.K = n;
    h.A = L;
    h.lda = n;
    h.outerA = (long long)mat;
    h.opA = 1;
    h.B = T;
    h.ldb = n;
    h.strideB = (long long)mat;
    h.opB = 0;
    h.C = B;
    h.ldc = n;
    h.strideC = (long long)mat;
    h.boff = b0;
    h.binner = nomega;
    h.alpha = 1.0;
    h.lower_only = 1;
    h.kmode = 2;
    h.skip = rboth;
    if (cplx) HIP_TRY(ctx, launch_zgemm(h, nb, s));
    DgemmArgs hr{};
    hr.M = hr.N = hr.K = n;
    hr.A = L;
    hr.lda = n;
    hr.outerA = (long long)mat;
    hr.opA = 1;
    hr.B = T + n2;
    hr.ldb = n;
    hr.strideB = (long long)mat;
    hr.C = B;
    hr.ldc = n;
    hr.strideC = (long long)mat;
    hr.boff = b0;
    hr.binner = nomega;
    hr.alpha = 1.0;
    hr.lower_only = 1;
    hr.kmode = 2;
    hr.sel = rboth;
    if (rl) HIP_TRY(ctx, launch_dgemm(hr, nb, s));
    const int *rp = rpair + b0;   // per matrix of the batch
    HIP_TRY(ctx, launch_trace_identity_minus(B, mat, n, nb, trB + b0, rp, s));
    HIP_TRY(ctx, launch_cholesky(B, mat, n, nb, W, flags, nq + b0, rp, s, kinds));
    HIP_TRY(ctx, launch_logdet(B, mat, n, nb, trB + b0, f + b0, flags, nq + b0, rp, s));
  }
  HIP_TRY(ctx, launch_quadrature(f, womega_dev, nq, nomega, ecq, s));
  return RPA_OK;
}

// The whole energy stage of one cell enqueued on stream s: kernels only (no host copy, no wait,
// no memset), so it can be captured into a graph; both kinds of q point are provided for.
// womega_dev: device [nomega].  Leaves the flags and per-q terms (ecq[q], ecq[nq] = E_c) in the
// workspace at l.flags and l.ecq.
int ec_enqueue(rpa_ctx *ctx, hipStream_t s, int n, int nq, int nomega, const double *womega_dev,
               const double *chi0_q, const double *v_q, char *ws, const EcLayout &l) {
  const int rc = ec_flags_enqueue(ctx, s, n, nq, nomega, chi0_q, v_q, ws, l);
  if (rc != RPA_OK) return rc;
  return ec_main_enqueue(ctx, s, n, nq, nomega, womega_dev, chi0_q, v_q, ws, l, 3);
}

// The energy stage for a caller that waits for it anyway: the kinds of q point present are read
// back after the flags (8 bytes, one wait), so the launches of an absent kind are left out.
int ec_enqueue_known(rpa_ctx *ctx, hipStream_t s, int n, int nq, int nomega, const double *womega_dev,
                     const double *chi0_q, const double *v_q, char *ws, const EcLayout &l) {
  int rc = ec_flags_enqueue(ctx, s, n, nq, nomega, chi0_q, v_q, ws, l);
  if (rc != RPA_OK) return rc;
  int counts[2] = {1, 1};
  HIP_TRY(ctx, hipMemcpyAsync(counts, ws + l.counts, sizeof(counts), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  const int kinds = (counts[1] > 0 ? 1 : 0) | (counts[0] > 0 ? 2 : 0);
  return ec_main_enqueue(ctx, s, n, nq, nomega, womega_dev, chi0_q, v_q, ws, l, kinds ? kinds : 3);
}

// phases exp(2 pi i q . n_R) for R -> q, the fractional part of q . n_R reduced before the 2 pi
std::vector<double> r2q_phases(const int mesh[3], int nq, const double *q_frac) {
  const int nR = mesh[0] * mesh[1] * mesh[2];
  std::vector<double> ph((size_t)2 * nq * nR);
  for (int q = 0; q < nq; ++q)
    for (int r = 0; r < nR; ++r) {
      const int n0 = r / (mesh[1] * mesh[2]), n1 = (r / mesh[2]) % mesh[1], n2 = r % mesh[2];
      double x = q_frac[3 * q] * n0 + q_frac[3 * q + 1] * n1 + q_frac[3 * q + 2] * n2;
      x -= std::floor(x);
      double c = std::cos(2.0 * M_PI * x), sn = std::sin(2.0 * M_PI * x);
      // quarter turns exactly (sin(pi) is not zero in floating point): chi(q) of a
      // time-reversal invariant q then comes out exactly real
      if (x == 0.0 || x == 0.25 || x == 0.5 || x == 0.75) {
        const int k = (int)(4.0 * x);
        c = k == 0 ? 1.0 : (k == 2 ? -1.0 : 0.0);
        sn = k == 1 ? 1.0 : (k == 3 ? -1.0 : 0.0);
      }
      ph[((size_t)q * nR + r) * 2] = c;
      ph[((size_t)q * nR + r) * 2 + 1] = sn;
    }
  return ph;
}
}  // namespace

// ---- batches of cells ----
struct BatchCell {
  rpa_batch_cell io;
  int n = 0, ntau = 0, nR = 0;
  size_t off_gamma = 0, off_ph = 0, off_w = 0;   // doubles into the batch's parameter buffer
  size_t off_flags = 0, off_ecq = 0;             // bytes into the batch's result buffer
  EcLayout el{};
};

struct rpa_batch {
  rpa_ctx *ctx = nullptr;
  int nlanes = 0;
  std::vector<BatchCell> cells;
  std::vector<hipStream_t> lanes;
  hipStream_t origin = nullptr;                  // the stream the graph is captured on
  std::vector<hipEvent_t> events;                // fork, then one join per lane
  double *dparams = nullptr;
  char *dres = nullptr;
  size_t res_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// The chi0 build in its steps.  T: precision of G, N and the N stage; bf16: split-BF16 fused
// kernel and, where the plan allows, split-BF16 N stage (T = float).  G is rescaled per tau
// by a power of two for the FP32 and BF16X3 paths; the fused kernel's epilogue removes it.
template <typename T>
struct BuildSteps {
  rpa_plan *p;
  rpa_ctx *ctx;
  hipStream_t s;
  char *ws;
  bool bf16, nbf;
  size_t gstride, chistride;
  T *Cp, *Gp, *Nb;
  uint16_t *Cb, *GTh, *GTl, *Cth, *Ctl;
  int *gexp;
  double *gpart;

  BuildSteps(rpa_plan *p_, char *ws_, bool bf16_) : p(p_), ctx(p_->ctx), s(p_->ctx->stream), ws(ws_), bf16(bf16_) {
    nbf = bf16 && p->nbf16;
    gstride = (size_t)p->nR * p->nb * p->nb;
    chistride = (size_t)p->nR * p->nauxtot * p->nauxtot;
    Cp = (T *)(ws + p->ws_cp);
    Cb = (uint16_t *)(ws + p->ws_cb);
    Gp = (T *)(ws + p->ws_g);
    Nb = (T *)(ws + p->ws_n);
    gpart = (double *)(ws + p->ws_sc);
    gexp = sizeof(T) == 4 ? (int *)(gpart + 2 * kGscaleBlocks) : nullptr;
    GTh = (uint16_t *)(ws + p->ws_gt);
    GTl = (uint16_t *)(ws + p->ws_gt + align_up(p->gt_bytes));
    Cth = (uint16_t *)(ws + p->ws_ct);
    Ctl = (uint16_t *)(ws + p->ws_ct + align_up(p->ct_bytes));
    Nsp = (uint16_t *)(ws + p->ws_ns);
  }
  uint16_t *Nsp;
  uint16_t *ns_at(int k) const { return (uint16_t *)((char *)Nsp + k * p->ns_slot); }
  // per-slot views
  T *gp_at(int k) const { return (T *)((char *)Gp + k * p->g_slot); }
  T *n_at(int k) const { return (T *)((char *)Nb + k * p->n_slot); }
  int *gexp_at(int k) const { return gexp ? gexp + 2 * k : nullptr; }
  int pack(const double *C) {
    Timed tm(ctx, "pack_c");
    if (nbf)
      HIP_TRY(ctx, launch_pack_ctn(p->pack, C, Cth, Ctl, p->maxblk, s));
    else
      HIP_TRY(ctx, launch_pack_c<T>(p->pack, C, Cp, p->maxblk, s));
    if (bf16) HIP_TRY(ctx, launch_pack_cb(p->pack, C, Cb, p->maxblk * 4, s));
    return RPA_OK;
  }
  // G of tau t into slot k
  int pad(const double *G_occ, const double *G_un, int t, int k = 0) {
    Timed tm(ctx, "pad_g");
    int *ge = gexp_at(k);
    if (ge) HIP_TRY(ctx, launch_gscale(G_occ + t * gstride, G_un + t * gstride, gstride, gpart, ge, s));
    HIP_TRY(ctx, launch_pad_g<T>(G_occ + t * gstride, G_un + t * gstride, p->nR, p->nb, p->nbp, ge, gp_at(k), s));
    if (nbf)
      HIP_TRY(ctx, launch_pad_gt(G_occ + t * gstride, G_un + t * gstride, p->nR, p->nb, p->nbp, p->nbq, p->dgsrc,
                                 ge, (uint16_t *)((char *)GTh + k * p->gt_slot),
                                 (uint16_t *)((char *)GTl + k * p->gt_slot), s));
    return RPA_OK;
  }
  // N of the first `ns` slots (one launch on the split-BF16 path, one per slot otherwise)
  int nstage(const rpa_tuning &tu, int ns = 1) {
    Timed tm(ctx, "nstage");
    const NTiles &tiles = p->ntiles(tu.nstage_order, nbf ? tu.nstage_bm : 128);
    if (nbf)
      HIP_TRY(ctx, launch_nstage_bf16(p->tb, tiles, tu.nstage_bm, GTh, GTl, p->gt_bytes, Cth, Ctl, p->ct_bytes,
                                      (float *)Nb, ns, p->gt_slot / sizeof(uint16_t), p->n_slot / sizeof(float), s));
    else
      for (int k = 0; k < ns; ++k)
        HIP_TRY(ctx, launch_nstage<T>(p->tb, tiles, gp_at(k), Cp, n_at(k), (size_t)p->cp_elems, tu.nstage_kstep, s));
    return RPA_OK;
  }
  // the split-BF16 copy of N that the split-BF16 fused kernel's O GEMM reads
  int split(int ns = 1) {
    if (!bf16) return RPA_OK;
    Timed tm(ctx, "split_n");
    HIP_TRY(ctx, launch_split_n(p->tb, (const float *)Nb, Nsp, ns, p->n_slot / sizeof(float),
                                p->ns_slot / sizeof(uint16_t), s));
    return RPA_OK;
  }
  // Screening bounds of tau t (when the plan screens).
  int screen(const double *G_occ, const double *G_un, int t, int k = 0) {
    if (p->theta <= 0.0) return RPA_OK;
    Timed tm(ctx, "screen");
    const size_t nb3 = (size_t)p->natoms * p->natoms * p->nR;
    HIP_TRY(ctx, launch_screen_norms(p->tb, G_occ + t * gstride, G_un + t * gstride, p->theta, p->scr_gb + k * nb3,
                                     p->scr_gn + k * nb3, p->scr_gc + 2 * k, s));
    return RPA_OK;
  }
  // chi of the first `ns` slots, slot k -> chi_t + k chistride.  stats_tau: tau of slot 0 for
  // the per-item screening statistics, or -1 for none.  The split-BF16 path runs either one
  // launch per template class and slot or, with tu.fused_single, one launch over every class
  // and slot (items in order of decreasing work).
  int fused(const rpa_tuning &tu, double negs, double *chi_t, int stats_tau = -1, int ns = 1) {
    Timed tm(ctx, "fused");
    const size_t nitems = p->itemU.size();
    const size_t nb3 = (size_t)p->natoms * p->natoms * p->nR;
    if (bf16 && tu.fused_single) {
      SingleLaunch a{};
      a.U = p->items.U;
      a.V = p->items.V;
      a.R = p->items.R;
      a.cls = p->d_item_cls;
      const bool halves = tu.fused_single == 2;
      a.order = halves ? p->d_half_order : p->d_item_order;
      a.nitems = halves ? (int)p->half_order.size() : (int)nitems;
      a.nslots = ns;
      a.Gp = (const float *)Gp;
      a.gp_stride = p->g_slot / sizeof(float);
      a.Cb = Cb;
      a.Nbuf = (const float *)Nb;
      a.n_stride = p->n_slot / sizeof(float);
      a.Ns = Nsp;
      a.ns_stride = p->ns_slot / sizeof(uint16_t);
      a.gexp = gexp;
      a.negs = negs;
      a.chi = chi_t;
      a.chi_stride = chistride;
      if (p->theta > 0.0) {
        a.gb = p->scr_gb;
        a.gn = p->scr_gn;
        a.gc = p->scr_gc;
        if (stats_tau >= 0) {
          a.stats = p->scr_stats + (size_t)stats_tau * nitems * 3;
          a.stats_stride = nitems * 3;
        }
      }
      HIP_TRY(ctx, launch_fused_bf16_single(p->tb, a, tu.fused_single, s));
      return RPA_OK;
    }
    for (int k = 0; k < ns; ++k)
      for (const PlanGroup &g : p->groups) {
        Screen sc{nullptr, nullptr, nullptr, nullptr};
        if (p->theta > 0.0) {
          sc = Screen{p->scr_gb + k * nb3, p->scr_gn + k * nb3, p->scr_gc + 2 * k, nullptr};
          if (stats_tau >= 0) sc.stats = p->scr_stats + ((size_t)(stats_tau + k) * nitems + g.start) * 3;
        }
        if (bf16)
          HIP_TRY(ctx, launch_fused_bf16(p->tb, p->group_items(g, tu.fused_order), g.mt, fused_bf16_ks_class(g.js),
                                         g.hc, (const float *)gp_at(k), Cb, (const float *)n_at(k), ns_at(k), negs,
                                         gexp_at(k), sc, chi_t + k * chistride, s));
        else
          HIP_TRY(ctx, launch_fused<T>(p->tb, p->group_items(g, tu.fused_order), g.mt, g.js, g.hc, gp_at(k), Cp,
                                       n_at(k), negs, gexp_at(k), sc, chi_t + k * chistride, s));
      }
    return RPA_OK;
  }
};

template <typename T>
static int build_impl(rpa_plan *p, const double *G_occ, const double *G_un, const double *C, char *ws, double negs,
                      double *chi0_tau, bool bf16) {
  BuildSteps<T> b(p, ws, bf16);
  int rc = b.pack(C);
  // tau points in chunks of p->slots: G of every tau of the chunk, then one N stage and the
  // fused kernel over the chunk
  for (int t0 = 0; rc == RPA_OK && t0 < p->ntau; t0 += p->slots) {
    const int ns = std::min(p->slots, p->ntau - t0);
    for (int k = 0; rc == RPA_OK && k < ns; ++k) {
      rc = b.pad(G_occ, G_un, t0 + k, k);
      if (rc == RPA_OK) rc = b.screen(G_occ, G_un, t0 + k, k);
    }
    if (rc == RPA_OK) rc = b.nstage(p->tune, ns);
    if (rc == RPA_OK) rc = b.split(ns);
    if (rc == RPA_OK) rc = b.fused(p->tune, negs, chi0_tau + t0 * b.chistride, t0, ns);
  }
  p->scr_valid = rc == RPA_OK && p->theta > 0.0;
  return rc;
}

// Autotuner: each candidate once untimed, once timed between two events on the stream; the plan
// defaults come first, and a later candidate replaces the best so far only when it is at least
// kTuneMargin faster (differences within the timing noise keep the default).
constexpr float kTuneMargin = 0.02f;
template <typename T>
static int autotune_impl(rpa_plan *p, const double *G_occ, const double *G_un, const double *C, char *ws, double negs,
                         double *chi_scratch, bool bf16, rpa_tuning &best) {
  rpa_ctx *ctx = p->ctx;
  BuildSteps<T> b(p, ws, bf16);
  int rc = b.pack(C);
  if (rc == RPA_OK) rc = b.pad(G_occ, G_un, 0);
  if (rc == RPA_OK) rc = b.screen(G_occ, G_un, 0);
  if (rc != RPA_OK) return rc;
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, RPA_ERR_HIP, "hipEventCreate failed");
  }
  auto timed = [&](auto &&step, float &ms) -> int {
    int r = step();
    if (r != RPA_OK) return r;
    if (hipEventRecord(e0, b.s) != hipSuccess) return fail(ctx, RPA_ERR_HIP, "hipEventRecord failed");
    r = step();
    if (r != RPA_OK) return r;
    if (hipEventRecord(e1, b.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return fail(ctx, RPA_ERR_HIP, "timing events failed");
    return RPA_OK;
  };
  best = p->tune;
  // N stage: tile order x K step (the split-BF16 N stage has no K-step choice)
  float tbest = 0.f;
  bool have = false;
  // N stage: tile order x K step (FP32 / FP64 N stage) or x tile rows (split-BF16 N stage)
  const int ksteps[2] = {16, 32}, bms[2] = {128, 256};
  for (int order = 0; rc == RPA_OK && order < 2; ++order)
    for (int ki = 0; rc == RPA_OK && ki < 2; ++ki) {
      rpa_tuning c = best;
      c.nstage_order = order;
      c.nstage_kstep = b.nbf ? 0 : ksteps[ki];
      c.nstage_bm = b.nbf ? bms[ki] : 128;
      float ms = 0.f;
      rc = timed([&]() { return b.nstage(c); }, ms);
      if (rc == RPA_OK && (!have || ms < (1.f - kTuneMargin) * tbest)) {
        tbest = ms;
        have = true;
        best.nstage_order = c.nstage_order;
        best.nstage_kstep = c.nstage_kstep;
        best.nstage_bm = c.nstage_bm;
        best.nstage_ms = ms;
      }
    }
  // fused kernel on the N of the chosen N stage
  if (rc == RPA_OK) rc = b.nstage(best);
  if (rc == RPA_OK) rc = b.split();
  // fused kernel: item order of the per-class launches, then (split BF16) the single launch
  have = false;
  for (int cand = 0; rc == RPA_OK && cand < (bf16 ? 5 : 2); ++cand) {
    rpa_tuning c = best;
    c.fused_order = cand == 1 ? 1 : 0;
    c.fused_single = cand >= 2 ? cand - 1 : 0;
    float ms = 0.f;
    rc = timed([&]() { return b.fused(c, negs, chi_scratch); }, ms);
    if (rc == RPA_OK && (!have || ms < (1.f - kTuneMargin) * tbest)) {
      tbest = ms;
      have = true;
      best.fused_order = c.fused_order;
      best.fused_single = c.fused_single;
      best.fused_ms = ms;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

// Workspace layout of a plan for p->slots tau points per launch: packed C (FP32 / FP64 N stage),
// split-BF16 C (BF16X3 fused kernel), then per slot padded G and N, the G scale (partial maxima,
// two exponents per slot), for the split-BF16 N stage transposed G per slot (hi and lo parts) and
// C (hi and lo), and on BF16X3 plans the split-BF16 copy of N per slot.
static void plan_layout(rpa_plan *p) {
  const size_t es = p->prec == RPA_FP64 ? 8 : 4;
  const int ns = p->slots;
  const size_t gtb = p->gt_bytes, ctb = p->ct_bytes;
  p->ws_cp = 0;
  p->ws_cb = align_up(p->nbf16 ? 0 : p->cp_elems * es);
  p->ws_g = align_up(p->ws_cb + (p->prec == RPA_BF16X3 ? (size_t)p->cb_elems * 2 : 0));
  p->g_slot = align_up(2 * (size_t)p->nR * p->nbp * p->nbp * es);
  p->ws_n = align_up(p->ws_g + ns * p->g_slot);
  p->n_slot = align_up((size_t)p->n_elems * es);
  p->ws_sc = align_up(p->ws_n + ns * p->n_slot);
  p->ws_gt = align_up(p->ws_sc + 2 * kGscaleBlocks * sizeof(double) + 2 * ns * sizeof(int));
  p->gt_slot = p->nbf16 ? 2 * align_up(gtb) : 0;
  p->ws_ct = align_up(p->ws_gt + ns * p->gt_slot);
  p->ws_ns = align_up(p->ws_ct + (p->nbf16 ? 2 * align_up(ctb) : 0));
  p->ns_slot = align_up((size_t)p->ns_elems * 2);
  p->ws_total = align_up(p->ws_ns + ns * p->ns_slot);
}

extern "C" {

int rpa_create(rpa_ctx **out, int device, void *hip_stream) {
  if (!out) return RPA_ERR_ARG;
  *out = nullptr;
  rpa_ctx *ctx = new rpa_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMalloc(&ctx->params, kParamsBytes);
  // once per device, with the device current: the address of its copy of the scratch array
  if (e == hipSuccess) e = scratch_setup(device, &ctx->scratch);
  if (e != hipSuccess) {
    if (ctx->params) hipFree(ctx->params);
    delete ctx;
    return RPA_ERR_HIP;
  }
  ctx->params_bytes = kParamsBytes;
  *out = ctx;
  return RPA_OK;
}

int rpa_set_stream(rpa_ctx *ctx, void *hip_stream) {
  if (!ctx) return RPA_ERR_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return RPA_OK;
}

void rpa_destroy(rpa_ctx *ctx) {
  if (!ctx) return;
  drain_profile(ctx);
  if (ctx->params) {
    hipStreamSynchronize(ctx->stream);
    hipFree(ctx->params);
  }
  delete ctx;
}

const char *rpa_last_error(const rpa_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int rpa_plan_create(rpa_ctx *ctx, const rpa_cell *cell, const rpa_lri_blocks *blocks, int ntau, int precision,
                    size_t *workspace_bytes, rpa_plan **out) {
  if (!ctx) return RPA_ERR_ARG;
  if (!cell || !blocks || !workspace_bytes || !out) return fail(ctx, RPA_ERR_ARG, "null argument");
  *out = nullptr;
  if (cell->natoms <= 0 || !cell->nao || !cell->naux) return fail(ctx, RPA_ERR_ARG, "bad cell");
  if (ntau <= 0) return fail(ctx, RPA_ERR_ARG, "ntau must be positive");
  if (precision != RPA_FP64 && precision != RPA_FP32 && precision != RPA_BF16X3)
    return fail(ctx, RPA_ERR_ARG, "unknown precision");
  for (int d = 0; d < 3; ++d) {
    if (cell->mesh[d] <= 0) return fail(ctx, RPA_ERR_ARG, "mesh must be positive");
    if (cell->mesh[d] > 1023) return fail(ctx, RPA_ERR_UNSUPPORTED, "mesh dimensions must be below 1024");
  }
  if (blocks->nblk < 0 || (blocks->nblk > 0 && (!blocks->I || !blocks->K || !blocks->R || !blocks->off)))
    return fail(ctx, RPA_ERR_ARG, "bad block list");

  rpa_plan *p = new rpa_plan();
  p->ctx = ctx;
  p->device = ctx->device;
  p->natoms = cell->natoms;
  p->ntau = ntau;
  p->prec = precision;
  for (int d = 0; d < 3; ++d) p->mesh[d] = cell->mesh[d];
  p->bvk = Bvk{cell->mesh[0], cell->mesh[1], cell->mesh[2]};
  p->nR = cell->mesh[0] * cell->mesh[1] * cell->mesh[2];
  const int na = p->natoms;
  p->nao.assign(cell->nao, cell->nao + na);
  p->naux.assign(cell->naux, cell->naux + na);
  for (int a = 0; a < na; ++a) {
    if (p->nao[a] <= 0 || p->naux[a] <= 0) {
      delete p;
      return fail(ctx, RPA_ERR_SHAPE, "nao and naux must be positive");
    }
    if (p->nao[a] > kMaxNao || p->naux[a] > kMaxNaux) {
      delete p;
      return fail(ctx, RPA_ERR_UNSUPPORTED, "nao <= 32 and naux <= 128 per atom in this build");
    }
  }
  p->ao_off.resize(na);
  p->aux_off.resize(na);
  for (int a = 0, o = 0, x = 0; a < na; ++a) {
    p->ao_off[a] = o;
    p->aux_off[a] = x;
    o += p->nao[a];
    x += p->naux[a];
  }
  p->nb = p->ao_off[na - 1] + p->nao[na - 1];
  p->nauxtot = p->aux_off[na - 1] + p->naux[na - 1];
  p->nbp = (p->nb + 7) / 8 * 8;
  p->cp_stride.resize(na);
  for (int a = 0; a < na; ++a) p->cp_stride[a] = (p->nao[a] * p->naux[a] + 7) / 8 * 8;
  p->atom_of_ao.resize(p->nb);
  for (int a = 0; a < na; ++a)
    for (int i = 0; i < p->nao[a]; ++i) p->atom_of_ao[p->ao_off[a] + i] = a;

  // blocks: validate, packed offsets (caller order), CSR by first atom (stable)
  const int nblk = blocks->nblk;
  p->nblk = nblk;
  p->in_off.resize(nblk);
  p->out_off.resize(nblk);
  p->cb_off.resize(nblk);
  p->ctn_off.resize(nblk);
  p->blk_a.resize(nblk);
  p->blk_ni.resize(nblk);
  p->blk_nk.resize(nblk);
  p->blk_stride.resize(nblk);
  std::vector<int> fR(nblk);
  long long acc = 0;
  for (int b = 0; b < nblk; ++b) {
    const int I = blocks->I[b], K = blocks->K[b];
    if (I < 0 || I >= na || K < 0 || K >= na || blocks->off[b] < 0) {
      delete p;
      return fail(ctx, RPA_ERR_SHAPE, "block atom index or offset out of range");
    }
    int f[3];
    for (int d = 0; d < 3; ++d) {
      const int m = cell->mesh[d];
      f[d] = ((blocks->R[3 * b + d] % m) + m) % m;
    }
    fR[b] = p->bvk.join(f[0], f[1], f[2]);
    p->in_off[b] = blocks->off[b];
    p->out_off[b] = acc;
    p->blk_a[b] = p->naux[I];
    p->blk_ni[b] = p->nao[I];
    p->blk_nk[b] = p->nao[K];
    p->blk_stride[b] = p->cp_stride[I];
    const long long sz = (long long)p->cp_stride[I] * p->nao[K];   // packed: [k][(i, mu)], padded rows
    p->maxblk = std::max(p->maxblk, sz);
    acc += sz;
    // split-BF16: [k][mu][hi, lo] rows of 2 x 16 hc slots
    p->cb_off[b] = p->cb_elems;
    p->cb_elems += (long long)p->nao[K] * p->naux[I] * 2 * 16 * (p->nao[I] > 16 ? 2 : 1);
    // split-BF16 N stage: [(i, mu)][k] with k padded to a multiple of 8
    p->ctn_off[b] = p->ctn_elems;
    p->ctn_elems += (long long)p->nao[I] * p->naux[I] * ((p->nao[K] + 7) / 8 * 8);
  }
  p->cp_elems = acc;
  p->nbr_start.assign(na + 1, 0);
  for (int b = 0; b < nblk; ++b) p->nbr_start[blocks->I[b] + 1]++;
  for (int a = 0; a < na; ++a) p->nbr_start[a + 1] += p->nbr_start[a];
  std::vector<int> order(nblk), fill(p->nbr_start.begin(), p->nbr_start.end() - 1);
  for (int b = 0; b < nblk; ++b) order[fill[blocks->I[b]]++] = b;
  // entries of one neighbourhood grouped by atom K (caller order kept within a group): the
  // fused kernels walk each group's periodic images together
  for (int a = 0; a < na; ++a)
    std::stable_sort(order.begin() + p->nbr_start[a], order.begin() + p->nbr_start[a + 1],
                     [&](int x, int y) { return blocks->K[x] < blocks->K[y]; });
  p->nbr_K.resize(nblk);
  p->nbr_R1.resize(nblk);
  p->nbr_cp.resize(nblk);
  p->nbr_cb.resize(nblk);
  for (int e = 0; e < nblk; ++e) {
    const int b = order[e];
    p->nbr_K[e] = blocks->K[b];
    p->nbr_R1[e] = fR[b];
    p->nbr_cp[e] = p->out_off[b];
    p->nbr_cb[e] = p->cb_off[b];
  }
  // end of the run of entries with the same atom K that holds entry e (the fused kernels' walk)
  p->nbr_run_end.resize(nblk);
  for (int a = 0; a < na; ++a)
    for (int e = p->nbr_start[a + 1] - 1; e >= p->nbr_start[a]; --e)
      p->nbr_run_end[e] = e + 1 < p->nbr_start[a + 1] && p->nbr_K[e + 1] == p->nbr_K[e] ? p->nbr_run_end[e + 1] : e + 1;
  p->nslices.assign(na, 0);
  for (int a = 0; a < na; ++a)
    for (int e = p->nbr_start[a]; e < p->nbr_start[a + 1]; ++e) p->nslices[a] += p->nao[p->nbr_K[e]];
  // N-stage contraction rows per atom V
  std::vector<long long> S(na, 0);
  p->rows_start.assign(na + 1, 0);
  for (int V = 0; V < na; ++V) {
    for (int e = p->nbr_start[V]; e < p->nbr_start[V + 1]; ++e) {
      const int L = p->nbr_K[e];
      S[V] += p->nao[L];
      int c0, c1, c2;
      p->bvk.split(p->nbr_R1[e], c0, c1, c2);
      for (int l = 0; l < p->nao[L]; ++l) {
        const long long cp = p->nbr_cp[e] + (long long)l * p->cp_stride[V];
        p->row_info.push_back(make_int4(p->ao_off[L] + l, c0 | (c1 << 10) | (c2 << 20), (int)(cp & 0xffffffffLL),
                                        (int)(cp >> 32)));
      }
    }
    p->rows_start[V + 1] = (int)p->row_info.size();
  }
  // split-BF16 N stage: GT columns padded per atom, contraction rows of V in groups of 8
  p->aopad_off.assign(na, 0);
  for (int a = 0; a < na; ++a) {
    p->aopad_off[a] = p->nbq;
    p->nbq += (p->nao[a] + 7) / 8 * 8;
  }
  p->gsrc.assign(p->nbq, -1);
  for (int a = 0; a < na; ++a)
    for (int i = 0; i < p->nao[a]; ++i) p->gsrc[p->aopad_off[a] + i] = p->ao_off[a] + i;
  p->ngrp_start.assign(na + 1, 0);
  for (int V = 0; V < na; ++V) {
    for (int e = p->nbr_start[V]; e < p->nbr_start[V + 1]; ++e) {
      const int b = order[e], L = p->nbr_K[e];
      const int st = (p->nao[L] + 7) / 8 * 8;
      int c0, c1, c2;
      p->bvk.split(p->nbr_R1[e], c0, c1, c2);
      for (int c = 0; c < st; c += 8) {
        p->ngrp.push_back(make_int4(p->aopad_off[L] + c, c0 | (c1 << 10) | (c2 << 20), st, 0));
        p->ngrp_off.push_back(p->ctn_off[b] + c);
      }
    }
    p->ngrp_start[V + 1] = (int)p->ngrp.size();
  }
  // N buffer offsets: block (V, K, dR) holds [k][s][j][nu]
  const int nR = p->nR;
  p->noff.resize((size_t)na * na * nR);
  long long no = 0;
  for (int V = 0; V < na; ++V)
    for (int K = 0; K < na; ++K)
      for (int r = 0; r < nR; ++r) {
        p->noff[((size_t)V * na + K) * nR + r] = no;
        no += (long long)p->nao[K] * 2 * p->nao[V] * p->naux[V];
      }
  p->n_elems = no;
  // split-BF16 copy of N: block (V, K, dR) holds [k][hi, lo][nu][2 n_V rounded up to 8]
  p->noffs.resize(p->noff.size());
  long long nso = 0;
  for (int V = 0; V < na; ++V)
    for (int K = 0; K < na; ++K)
      for (int r = 0; r < nR; ++r) {
        p->noffs[((size_t)V * na + K) * nR + r] = nso;
        nso += (long long)p->nao[K] * 2 * p->naux[V] * ((2 * p->nao[V] + 7) / 8 * 8);
      }
  p->ns_elems = precision == RPA_BF16X3 ? nso : 0;
  // N-stage tiles of each atom V in blocks of 8 column tiles by 8 row tiles (by 4 for the
  // 256-row tiles): the 64 workgroups one XCD runs at a time then share 8 B column tiles and 8
  // A row tiles in its L2, where a column of row tiles shares only its B tile
  const int M = 2 * nR * p->nbp;
  for (int V = 0; V < na; ++V) {
    const int NV = p->nao[V] * p->naux[V];
    for (int nb0 = 0; nb0 < NV; nb0 += 8 * 128)
      for (int mb0 = 0; mb0 < M; mb0 += 8 * 128)
        for (int n0 = nb0; n0 < std::min(NV, nb0 + 8 * 128); n0 += 128)
          for (int m0 = mb0; m0 < std::min(M, mb0 + 8 * 128); m0 += 128) {
            p->tileV.push_back(V);
            p->tileM.push_back(m0);
            p->tileN.push_back(n0);
          }
    for (int nb0 = 0; nb0 < NV; nb0 += 8 * 128)
      for (int mb0 = 0; mb0 < M; mb0 += 4 * 256)
        for (int n0 = nb0; n0 < std::min(NV, nb0 + 8 * 128); n0 += 128)
          for (int m0 = mb0; m0 < std::min(M, mb0 + 4 * 256); m0 += 256) {
            p->tile2V.push_back(V);
            p->tile2M.push_back(m0);
            p->tile2N.push_back(n0);
          }
  }
  // fused items: atom pairs U <= V (Sec. 3.2 pair set), all R; grouped by the kernel's
  // template classes (mu-tiles of U, O-GEMM steps of V)
  {
    std::map<std::tuple<int, int, int>, std::vector<std::pair<int, int>>> groups;
    for (int U = 0; U < na; ++U)
      for (int V = U; V < na; ++V)
        groups[{fused_mt_class(p->naux[U]), fused_js_class(p->nao[V]), p->nao[U] > 16 ? 2 : 1}].push_back({U, V});
    for (auto &g : groups) {
      PlanGroup pg;
      pg.mt = std::get<0>(g.first);
      pg.js = std::get<1>(g.first);
      pg.hc = std::get<2>(g.first);
      pg.start = (int)p->itemU.size();
      for (auto &uv : g.second)
        for (int r = 0; r < nR; ++r) {
          p->itemU.push_back(uv.first);
          p->itemV.push_back(uv.second);
          p->itemR.push_back(r);
        }
      pg.count = (int)p->itemU.size() - pg.start;
      p->groups.push_back(pg);
    }
  }
  // class code and work estimate of every item for the single fused launch: K(R1) slices of U
  // times the MFMA work of one slice in the item's class, plus the Z contraction; the list runs
  // from the largest item down, so the last workgroups of a launch take the smallest items
  {
    const size_t ni = p->itemU.size();
    p->item_cls.assign(ni, 0);
    std::vector<double> cost(ni, 0.0);
    for (const PlanGroup &g : p->groups) {
      const int ks = fused_bf16_ks_class(g.js);
      for (int i = g.start; i < g.start + g.count; ++i) {
        p->item_cls[i] = single_class(g.mt, ks, g.hc);
        const int U = p->itemU[i], V = p->itemV[i];
        cost[i] = (double)p->nslices[U] * (ks * g.hc + g.mt * g.hc) + 0.25 * p->nao[U] * p->nao[V] * g.mt;
      }
    }
    p->item_order.resize(ni);
    for (size_t i = 0; i < ni; ++i) p->item_order[i] = (int)i;
    std::stable_sort(p->item_order.begin(), p->item_order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    // 4-wave units: the first 64 ABF columns of V, and the rest where V has more
    for (int i : p->item_order) {
      p->half_order.push_back(2 * i);
      if (p->naux[p->itemV[i]] > 64) p->half_order.push_back(2 * i + 1);
    }
    std::stable_sort(p->half_order.begin(), p->half_order.end(), [&](int x, int y) {
      const double cx = cost[x >> 1] * (p->naux[p->itemV[x >> 1]] > 64 ? 0.5 : 1.0);
      const double cy = cost[y >> 1] * (p->naux[p->itemV[y >> 1]] > 64 ? 0.5 : 1.0);
      return cx > cy;
    });
  }
  for (int a = 0; a < na; ++a)
    if (p->nbr_start[a + 1] - p->nbr_start[a] > kMaxNbr) {
      delete p;
      return fail(ctx, RPA_ERR_UNSUPPORTED, "more than 1024 LRI blocks for one atom");
    }
  // XCD-grouped copies of the tile list and of each group's items
  std::vector<int> tileVx, tileMx, tileNx, itemUx, itemVx, itemRx, tile2Vx, tile2Mx, tile2Nx;
  {
    const std::vector<int> pt = xcd_grouped_order((int)p->tileV.size());
    for (int b : pt) {
      tileVx.push_back(p->tileV[b]);
      tileMx.push_back(p->tileM[b]);
      tileNx.push_back(p->tileN[b]);
    }
    for (int b : xcd_grouped_order((int)p->tile2V.size())) {
      tile2Vx.push_back(p->tile2V[b]);
      tile2Mx.push_back(p->tile2M[b]);
      tile2Nx.push_back(p->tile2N[b]);
    }
    itemUx.resize(p->itemU.size());
    itemVx.resize(p->itemU.size());
    itemRx.resize(p->itemU.size());
    for (const PlanGroup &g : p->groups) {
      const std::vector<int> pi = xcd_grouped_order(g.count);
      for (int b = 0; b < g.count; ++b) {
        itemUx[g.start + b] = p->itemU[g.start + pi[b]];
        itemVx[g.start + b] = p->itemV[g.start + pi[b]];
        itemRx[g.start + b] = p->itemR[g.start + pi[b]];
      }
    }
  }
  // autotuner shape class: everything the launch shapes and work lists depend on
  {
    std::string k = "p" + std::to_string(precision) + " na" + std::to_string(na) + " nb" + std::to_string(p->nb) +
                    " naux" + std::to_string(p->nauxtot) + " nR" + std::to_string(nR) + " blk" + std::to_string(nblk) +
                    " tiles" + std::to_string(p->tileV.size());
    for (const PlanGroup &g : p->groups)
      k += " g" + std::to_string(g.mt) + "." + std::to_string(g.js) + "." + std::to_string(g.hc) + "." +
           std::to_string(g.count);
    p->shape_key = k;
  }
  // flop model (per tau, times ntau)
  double fN = 0, fX = 0, fMZ = 0, fChi = 0, eN = 0, eFused = 0;
  for (int V = 0; V < na; ++V) fN += 2.0 * nR * 2.0 * p->naux[V] * p->nao[V] * p->nb * (double)S[V];
  eN = fN;
  for (int U = 0; U < na; ++U)
    for (int V = U; V < na; ++V) {
      const double nU = p->nao[U], aU = p->naux[U], nV = p->nao[V], aV = p->naux[V];
      fX += 2.0 * nR * 2.0 * nU * aV * nV * (double)S[V];
      fMZ += nR * 8.0 * nU * nV * aV * (double)S[U];
      fChi += nR * 2.0 * aU * aV * nU * (double)S[U];
      eFused += nR * (2.0 * nU * 2.0 * nV * aV * (double)S[U] + 2.0 * aU * aV * nU * (double)S[U] +
                      2.0 * aU * aV * 2.0 * nU * nV);
    }
  p->alg_flops = ntau * (fN + fX + fMZ + fChi);
  p->exec_flops = ntau * (eN + eFused);
  p->stage_alg[0] = ntau * fN;
  p->stage_alg[1] = ntau * (fX + fMZ + fChi);
  p->stage_exec[0] = ntau * eN;
  p->stage_exec[1] = ntau * eFused;

  // device tables: one allocation, 256-byte aligned sections
  struct Sec {
    const void *src;
    size_t bytes;
    size_t off;
  };
  std::vector<Sec> secs;
  size_t tot = 0;
  auto add = [&](const void *src, size_t bytes) {
    secs.push_back({src, bytes, tot});
    tot = align_up(tot + std::max<size_t>(bytes, 1));
    return secs.size() - 1;
  };
  const size_t s_nao = add(p->nao.data(), na * 4), s_naux = add(p->naux.data(), na * 4),
               s_aoo = add(p->ao_off.data(), na * 4), s_auxo = add(p->aux_off.data(), na * 4),
               s_aoa = add(p->atom_of_ao.data(), p->nb * 4), s_ns = add(p->nbr_start.data(), (na + 1) * 4),
               s_nK = add(p->nbr_K.data(), nblk * 4), s_nR1 = add(p->nbr_R1.data(), nblk * 4),
               s_nre = add(p->nbr_run_end.data(), nblk * 4),
               s_ncp = add(p->nbr_cp.data(), nblk * 8), s_rs = add(p->rows_start.data(), (na + 1) * 4),
               s_ri = add(p->row_info.data(), p->row_info.size() * 16), s_noff = add(p->noff.data(), p->noff.size() * 8),
               s_noffs = add(p->noffs.data(), p->noffs.size() * 8),
               s_tV = add(p->tileV.data(), p->tileV.size() * 4), s_tM = add(p->tileM.data(), p->tileM.size() * 4),
               s_tN = add(p->tileN.data(), p->tileN.size() * 4), s_iU = add(p->itemU.data(), p->itemU.size() * 4),
               s_iV = add(p->itemV.data(), p->itemV.size() * 4), s_iR = add(p->itemR.data(), p->itemR.size() * 4),
               s_pin = add(p->in_off.data(), nblk * 8), s_pout = add(p->out_off.data(), nblk * 8),
               s_pa = add(p->blk_a.data(), nblk * 4), s_pni = add(p->blk_ni.data(), nblk * 4),
               s_pnk = add(p->blk_nk.data(), nblk * 4), s_pst = add(p->blk_stride.data(), nblk * 4),
               s_cst = add(p->cp_stride.data(), na * 4), s_nsl = add(p->nslices.data(), na * 4),
               s_ncb = add(p->nbr_cb.data(), nblk * 8), s_pcb = add(p->cb_off.data(), nblk * 8),
               s_pct = add(p->ctn_off.data(), nblk * 8), s_gsrc = add(p->gsrc.data(), p->gsrc.size() * 4),
               s_ngs = add(p->ngrp_start.data(), (na + 1) * 4), s_ng = add(p->ngrp.data(), p->ngrp.size() * 16),
               s_ngo = add(p->ngrp_off.data(), p->ngrp_off.size() * 8);
  const size_t s_icls = add(p->item_cls.data(), p->item_cls.size() * 4),
               s_iord = add(p->item_order.data(), p->item_order.size() * 4),
               s_hord = add(p->half_order.data(), p->half_order.size() * 4);
  const size_t s_t2V = add(p->tile2V.data(), p->tile2V.size() * 4), s_t2M = add(p->tile2M.data(), p->tile2M.size() * 4),
               s_t2N = add(p->tile2N.data(), p->tile2N.size() * 4), s_t2Vx = add(tile2Vx.data(), tile2Vx.size() * 4),
               s_t2Mx = add(tile2Mx.data(), tile2Mx.size() * 4), s_t2Nx = add(tile2Nx.data(), tile2Nx.size() * 4);
  const size_t s_tVx = add(tileVx.data(), tileVx.size() * 4), s_tMx = add(tileMx.data(), tileMx.size() * 4),
               s_tNx = add(tileNx.data(), tileNx.size() * 4), s_iUx = add(itemUx.data(), itemUx.size() * 4),
               s_iVx = add(itemVx.data(), itemVx.size() * 4), s_iRx = add(itemRx.data(), itemRx.size() * 4);
  hipError_t he = table_alloc(ctx->device, &p->dtab, tot);
  if (he != hipSuccess) {
    delete p;
    return fail(ctx, RPA_ERR_HIP, std::string("plan tables: ") + hipGetErrorString(he));
  }
  std::vector<char> host(tot, 0);
  for (auto &s : secs)
    if (s.bytes) std::memcpy(host.data() + s.off, s.src, s.bytes);
  he = table_upload(p->dtab, host.data(), tot);
  if (he != hipSuccess) {
    table_free(ctx->device, p->dtab);
    delete p;
    return fail(ctx, RPA_ERR_HIP, std::string("plan tables copy: ") + hipGetErrorString(he));
  }
  char *d = (char *)p->dtab;
  auto I32 = [&](size_t s) { return (const int *)(d + secs[s].off); };
  auto I64 = [&](size_t s) { return (const long long *)(d + secs[s].off); };
  Chi0Tables &tb = p->tb;
  tb.nao = I32(s_nao);
  tb.naux = I32(s_naux);
  tb.ao_off = I32(s_aoo);
  tb.aux_off = I32(s_auxo);
  tb.atom_of_ao = I32(s_aoa);
  tb.nbr_start = I32(s_ns);
  tb.nbr_K = I32(s_nK);
  tb.nbr_R1 = I32(s_nR1);
  tb.nbr_run_end = I32(s_nre);
  tb.nbr_cp = I64(s_ncp);
  tb.rows_start = I32(s_rs);
  tb.row_info = (const int4 *)(d + secs[s_ri].off);
  tb.noff = I64(s_noff);
  tb.noffs = I64(s_noffs);
  tb.cp_stride = I32(s_cst);
  tb.nslices = I32(s_nsl);
  tb.nbr_cb = I64(s_ncb);
  tb.ngrp_start = I32(s_ngs);
  tb.ngrp = (const int4 *)(d + secs[s_ng].off);
  tb.ngrp_off = I64(s_ngo);
  tb.nbq = p->nbq;
  p->dgsrc = I32(s_gsrc);
  tb.natoms = na;
  tb.nb = p->nb;
  tb.nbp = p->nbp;
  tb.nauxtot = p->nauxtot;
  tb.nR = nR;
  tb.bvk = p->bvk;
  p->tiles = NTiles{I32(s_tV), I32(s_tM), I32(s_tN), (int)p->tileV.size()};
  p->items = PairItems{I32(s_iU), I32(s_iV), I32(s_iR), (int)p->itemU.size()};
  p->tiles_x = NTiles{I32(s_tVx), I32(s_tMx), I32(s_tNx), (int)tileVx.size()};
  p->tiles2 = NTiles{I32(s_t2V), I32(s_t2M), I32(s_t2N), (int)p->tile2V.size()};
  p->tiles2_x = NTiles{I32(s_t2Vx), I32(s_t2Mx), I32(s_t2Nx), (int)tile2Vx.size()};
  p->items_x = PairItems{I32(s_iUx), I32(s_iVx), I32(s_iRx), (int)itemUx.size()};
  p->pack = PackTables{I64(s_pin), I64(s_pout), I64(s_pcb), I64(s_pct), I32(s_pa), I32(s_pni), I32(s_pnk), I32(s_pst),
                       nblk};
  p->d_item_cls = I32(s_icls);
  p->d_item_order = I32(s_iord);
  p->d_half_order = I32(s_hord);


  // workspace: packed C (FP32 / FP64 N stage), split-BF16 C (BF16X3 fused kernel), padded G of
  // one tau, N buffer for one tau, G scale (partial maxima and the two exponents), and for the
  // split-BF16 N stage transposed G of one tau and C, hi and lo parts each
  const size_t kViewMax = (size_t)0xffff0000u;
  const size_t gtb = (size_t)2 * nR * p->nbp * p->nbq * 2, ctb = (size_t)p->ctn_elems * 2;
  p->nbf16 = precision == RPA_BF16X3 && gtb <= kViewMax && ctb <= kViewMax;
  p->gt_bytes = p->nbf16 ? (unsigned)gtb : 0u;
  p->ct_bytes = p->nbf16 ? (unsigned)ctb : 0u;
  p->tune.nstage_kstep = p->nbf16 ? 0 : 16;
  plan_layout(p);
  *workspace_bytes = p->ws_total;
  *out = p;
  return RPA_OK;
}

int rpa_plan_destroy(rpa_plan *p) {
  if (!p) return RPA_ERR_ARG;
  if (p->dscr) {
    // the buffer may still be read by queued kernels of this plan
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->dscr);
  }
  if (p->dtab) table_free(p->device, p->dtab);
  delete p;
  return RPA_OK;
}

// Screening buffer for p->slots tau points: bounds gb, gn and (g, cut) per slot, statistics of
// every tau.  Waits for the device before freeing an older buffer.
static int screen_alloc(rpa_plan *p) {
  const size_t nb3 = (size_t)p->natoms * p->natoms * p->nR;
  const size_t b_gb = align_up(p->slots * nb3 * sizeof(double)), b_gc = align_up(2 * p->slots * sizeof(double));
  const size_t b_st = align_up((size_t)p->ntau * p->itemU.size() * 3 * sizeof(int));
  HIP_TRY(p->ctx, hipSetDevice(p->device));
  if (p->dscr) {
    HIP_TRY(p->ctx, hipDeviceSynchronize());
    HIP_TRY(p->ctx, hipFree(p->dscr));
    p->dscr = nullptr;
  }
  HIP_TRY(p->ctx, hipMalloc(&p->dscr, 2 * b_gb + b_gc + b_st));
  char *d = (char *)p->dscr;
  p->scr_gb = (double *)d;
  p->scr_gn = (double *)(d + b_gb);
  p->scr_gc = (double *)(d + 2 * b_gb);
  p->scr_stats = (int *)(d + 2 * b_gb + b_gc);
  return RPA_OK;
}

int rpa_plan_set_screening(rpa_plan *p, double theta) {
  if (!p) return RPA_ERR_ARG;
  if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(p->ctx, RPA_ERR_ARG, "theta must be finite and >= 0");
  if (theta > 0.0 && !p->dscr) {
    const int rc = screen_alloc(p);
    if (rc != RPA_OK) return rc;
  }
  p->theta = theta;
  p->scr_valid = false;
  return RPA_OK;
}

int rpa_plan_set_tau_batch(rpa_plan *p, int ntau_per_launch, size_t *workspace_bytes) {
  if (!p) return RPA_ERR_ARG;
  if (!workspace_bytes) return fail(p->ctx, RPA_ERR_ARG, "null argument");
  if (ntau_per_launch < 1 || ntau_per_launch > p->ntau)
    return fail(p->ctx, RPA_ERR_ARG, "tau points per launch must be in [1, ntau]");
  p->slots = ntau_per_launch;
  plan_layout(p);
  if (p->dscr) {
    const int rc = screen_alloc(p);
    if (rc != RPA_OK) return rc;
  }
  p->scr_valid = false;
  *workspace_bytes = p->ws_total;
  return RPA_OK;
}

int rpa_plan_workspace_bytes(const rpa_plan *p, size_t *workspace_bytes) {
  if (!p || !workspace_bytes) return RPA_ERR_ARG;
  *workspace_bytes = p->ws_total;
  return RPA_OK;
}

int rpa_plan_screening_stats(rpa_plan *p, long long *out) {
  if (!p) return RPA_ERR_ARG;
  if (!out) return fail(p->ctx, RPA_ERR_ARG, "null argument");
  if (!p->scr_valid) return fail(p->ctx, RPA_ERR_ARG, "no screened build since the threshold was set");
  const size_t nitems = p->itemU.size();
  std::vector<int> h((size_t)p->ntau * nitems * 3);
  HIP_TRY(p->ctx, hipSetDevice(p->device));
  HIP_TRY(p->ctx, hipStreamSynchronize(p->ctx->stream));
  HIP_TRY(p->ctx, hipMemcpy(h.data(), p->scr_stats, h.size() * sizeof(int), hipMemcpyDeviceToHost));
  long long ek = 0, sk = 0, zk = 0, et = 0, st = 0;
  for (size_t i = 0; i < h.size(); i += 3) {
    ek += h[i];
    sk += h[i + 1];
    zk += h[i + 2];
  }
  for (size_t i = 0; i < nitems; ++i) {
    const int U = p->itemU[i];
    et += p->nbr_start[U + 1] - p->nbr_start[U];
    st += p->nslices[U];
  }
  out[0] = ek;
  out[1] = et * p->ntau;
  out[2] = sk;
  out[3] = st * p->ntau;
  out[4] = zk;
  out[5] = (long long)nitems * p->ntau;
  return RPA_OK;
}

int rpa_plan_flops(const rpa_plan *p, double *alg, double *exec) {
  if (!p || !alg || !exec) return RPA_ERR_ARG;
  *alg = p->alg_flops;
  *exec = p->exec_flops;
  return RPA_OK;
}

static bool tuning_valid(const rpa_plan *p, const rpa_tuning &t) {
  if (t.nstage_order != 0 && t.nstage_order != 1) return false;
  if (t.fused_order != 0 && t.fused_order != 1) return false;
  if (t.fused_single != 0 && !(t.fused_single >= 1 && t.fused_single <= 3 && p->prec == RPA_BF16X3)) return false;
  if (t.nstage_bm != 128 && !(t.nstage_bm == 256 && p->nbf16)) return false;
  return p->nbf16 ? t.nstage_kstep == 0 : (t.nstage_kstep == 16 || t.nstage_kstep == 32);
}

int rpa_plan_get_tuning(const rpa_plan *p, rpa_tuning *out) {
  if (!p || !out) return RPA_ERR_ARG;
  *out = p->tune;
  return RPA_OK;
}

int rpa_plan_set_tuning(rpa_plan *p, const rpa_tuning *t) {
  if (!p) return RPA_ERR_ARG;
  if (!t) return fail(p->ctx, RPA_ERR_ARG, "null tuning");
  if (!tuning_valid(p, *t))
    return fail(p->ctx, RPA_ERR_ARG,
                "tuning out of range (orders 0 or 1; K step 16 or 32, 0 for the split-BF16 N stage; single fused "
                "launch 0, or 1 or 2 on split-BF16 plans; N-stage tile rows 128, or 256 for the split-BF16 N stage)");
  p->tune = rpa_tuning{t->nstage_order, t->nstage_kstep, t->fused_order, 0, 0.0, 0.0, t->fused_single, t->nstage_bm};
  return RPA_OK;
}

int rpa_plan_autotune(rpa_plan *p, double spin_factor, const double *G_occ, const double *G_un, const double *C,
                      void *workspace, size_t workspace_bytes, double *chi0_scratch, rpa_tuning *out) {
  if (!p) return RPA_ERR_ARG;
  rpa_ctx *ctx = p->ctx;
  if (!G_occ || !G_un || !chi0_scratch || !workspace || (p->nblk > 0 && !C))
    return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (workspace_bytes < p->ws_total)
    return fail(ctx, RPA_ERR_WORKSPACE, "workspace smaller than rpa_plan_create reported");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipDeviceProp_t prop;
  HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
  const std::string key = std::string(prop.gcnArchName) + " " + p->shape_key;
  auto hit = ctx->tune_cache.find(key);
  if (hit != ctx->tune_cache.end() && tuning_valid(p, hit->second)) {
    p->tune = hit->second;
    p->tune.from_cache = 1;
    p->tune.nstage_ms = p->tune.fused_ms = 0.0;
  } else {
    rpa_tuning best{};
    const double negs = -spin_factor;
    const int rc = p->prec == RPA_FP64
                       ? autotune_impl<double>(p, G_occ, G_un, C, (char *)workspace, negs, chi0_scratch, false, best)
                       : autotune_impl<float>(p, G_occ, G_un, C, (char *)workspace, negs, chi0_scratch,
                                              p->prec == RPA_BF16X3, best);
    if (rc != RPA_OK) return rc;
    best.from_cache = 0;
    p->tune = best;
    ctx->tune_cache[key] = best;
  }
  if (out) *out = p->tune;
  return RPA_OK;
}

int rpa_plan_stage_flops(const rpa_plan *p, int stage, double *alg, double *exec) {
  if (!p || !alg || !exec || stage < 0 || stage > 1) return RPA_ERR_ARG;
  *alg = p->stage_alg[stage];
  *exec = p->stage_exec[stage];
  return RPA_OK;
}

int rpa_profile(rpa_ctx *ctx, int enable) {
  if (!ctx) return RPA_ERR_ARG;
  int rc = drain_profile(ctx);
  ctx->totals.clear();
  ctx->profile = enable != 0;
  return rc;
}

int rpa_profile_read(rpa_ctx *ctx, const char *kernel, double *total_ms, int *launches) {
  if (!ctx || !kernel || !total_ms || !launches) return RPA_ERR_ARG;
  if (drain_profile(ctx) != RPA_OK) return fail(ctx, RPA_ERR_HIP, "event timing failed");
  auto it = ctx->totals.find(kernel);
  *total_ms = it == ctx->totals.end() ? 0.0 : it->second.first;
  *launches = it == ctx->totals.end() ? 0 : it->second.second;
  return RPA_OK;
}

int build_chi0_tau(rpa_plan *p, double spin_factor, const double *G_occ, const double *G_un, const double *C,
                   void *workspace, size_t workspace_bytes, double *chi0_tau) {
  if (!p) return RPA_ERR_ARG;
  rpa_ctx *ctx = p->ctx;
  if (!G_occ || !G_un || !chi0_tau || !workspace || (p->nblk > 0 && !C))
    return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (workspace_bytes < p->ws_total)
    return fail(ctx, RPA_ERR_WORKSPACE, "workspace smaller than rpa_plan_create reported");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  char *ws = (char *)workspace;
  const double negs = -spin_factor;
  if (p->prec == RPA_FP64) return build_impl<double>(p, G_occ, G_un, C, ws, negs, chi0_tau, false);
  return build_impl<float>(p, G_occ, G_un, C, ws, negs, chi0_tau, p->prec == RPA_BF16X3);
}

int chi0_tau_to_omega(rpa_ctx *ctx, int ntau, int nomega, size_t n, const double *gamma_cos,
                      const double *chi0_tau, double *chi0_omega) {
  if (!ctx) return RPA_ERR_ARG;
  if (!gamma_cos || !chi0_tau || !chi0_omega) return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (ntau <= 0 || nomega <= 0 || ntau > 64 || nomega > 64)
    return fail(ctx, RPA_ERR_ARG, "ntau and nomega must be in [1, 64]");
  if (n == 0) return RPA_OK;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->params, gamma_cos, sizeof(double) * ntau * nomega, hipMemcpyHostToDevice,
                              ctx->stream));
  Timed tm(ctx, "cos_transform");
  HIP_TRY(ctx, launch_cos_transform(ctx->params, ntau, nomega, n, chi0_tau, chi0_omega, ctx->stream));
  return RPA_OK;
}

int chi0_R_to_q(rpa_ctx *ctx, const int mesh[3], int nbatch, size_t m, int nq, const double *q_frac,
                const double *chi0_R, double *chi0_q) {
  if (!ctx) return RPA_ERR_ARG;
  if (!mesh || !q_frac || !chi0_R || !chi0_q) return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (nbatch <= 0 || nq <= 0 || mesh[0] <= 0 || mesh[1] <= 0 || mesh[2] <= 0)
    return fail(ctx, RPA_ERR_ARG, "sizes must be positive");
  const int nR = mesh[0] * mesh[1] * mesh[2];
  if ((size_t)2 * nq * nR * sizeof(double) > 64 * 1024)
    return fail(ctx, RPA_ERR_UNSUPPORTED, "nq * nR must not exceed 4096");
  if (m == 0) return RPA_OK;
  const std::vector<double> ph = r2q_phases(mesh, nq, q_frac);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->params, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  Timed tm(ctx, "r2q");
  HIP_TRY(ctx, launch_r2q(ctx->params, nR, nq, nbatch, m, chi0_R, chi0_q, ctx->stream));
  return RPA_OK;
}


// Green's functions: workspace = X (complex [nk][nb][max band count]) + W (complex [nk][nb][nb])
static void green_layout(int nk, int nb, int nocc, size_t &x_bytes, size_t &total) {
  const size_t nbs = (size_t)std::max(nocc, nb - nocc);
  x_bytes = align_up((size_t)nk * nb * nbs * 16);
  total = x_bytes + align_up((size_t)nk * nb * nb * 16);
}

size_t rpa_green_workspace_size(int nk, int nb, int nocc) {
  if (nk <= 0 || nb <= 0 || nocc < 0 || nocc > nb) return 0;
  size_t x, t;
  green_layout(nk, nb, nocc, x, t);
  return t;
}

int build_green_tau(rpa_ctx *ctx, int nk, int nb, int nocc, double mu, int ntau, const double *tau, const int mesh[3],
                    const double *k_frac, const double *eps, const double *wfc, void *workspace,
                    size_t workspace_bytes, double *G_occ, double *G_un) {
  if (!ctx) return RPA_ERR_ARG;
  if (!tau || !mesh || !k_frac || !eps || !wfc || !workspace || !G_occ || !G_un)
    return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (nk <= 0 || nb <= 0 || ntau <= 0 || nocc < 0 || nocc > nb || mesh[0] <= 0 || mesh[1] <= 0 || mesh[2] <= 0)
    return fail(ctx, RPA_ERR_ARG, "need nk, nb, ntau, mesh > 0 and 0 <= nocc <= nb");
  const int nR = mesh[0] * mesh[1] * mesh[2];
  if ((long long)nR * nk > 4096) return fail(ctx, RPA_ERR_UNSUPPORTED, "nR * nk must not exceed 4096");
  size_t xb, total;
  green_layout(nk, nb, nocc, xb, total);
  if (workspace_bytes < total) return fail(ctx, RPA_ERR_WORKSPACE, "workspace smaller than rpa_green_workspace_size");
  // phases e^{-i k.R} / N_k, [nR][nk] complex
  std::vector<double> ph((size_t)2 * nR * nk);
  for (int r = 0; r < nR; ++r) {
    const int n3 = r % mesh[2], n2 = (r / mesh[2]) % mesh[1], n1 = r / (mesh[1] * mesh[2]);
    for (int k = 0; k < nk; ++k) {
      const double a = -2.0 * M_PI * (k_frac[3 * k] * n1 + k_frac[3 * k + 1] * n2 + k_frac[3 * k + 2] * n3);
      ph[((size_t)r * nk + k) * 2] = std::cos(a) / nk;
      ph[((size_t)r * nk + k) * 2 + 1] = std::sin(a) / nk;
    }
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->params, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice, s));
  double *X = (double *)workspace, *W = (double *)((char *)workspace + xb);
  const size_t m = (size_t)nb * nb, gstride = (size_t)nR * m;
  Timed tm(ctx, "green");
  for (int t = 0; t < ntau; ++t)
    for (int occ = 1; occ >= 0; --occ) {
      const int n0 = occ ? 0 : nocc, nbs = occ ? nocc : nb - nocc;
      HIP_TRY(ctx, launch_green_weight(eps, wfc, nk, nb, n0, nbs, mu, tau[t], occ, X, s));
      // W_k = X_k c_k[:, n0:n0+nbs]^H for every k (an empty band set gives W = 0)
      ZgemmArgs g{};
      g.M = g.N = nb;
      g.K = nbs;
      g.A = X;
      g.lda = nbs;
      g.strideA = (long long)nb * nbs * 2;
      g.opA = 0;
      g.B = wfc + 2 * (size_t)n0;
      g.ldb = nb;
      g.strideB = (long long)m * 2;
      g.opB = 1;
      g.C = W;
      g.ldc = nb;
      g.strideC = (long long)m * 2;
      g.alpha = 1.0;
      HIP_TRY(ctx, launch_zgemm(g, nk, s));
      HIP_TRY(ctx, launch_k2r_real(ctx->params, nR, nk, m, W, (occ ? G_occ : G_un) + t * gstride, s));
    }
  return RPA_OK;
}

int rpa_check_green_symmetry(rpa_ctx *ctx, int ntau, const int mesh[3], int nb, const double *G_occ,
                             const double *G_un, double tol, double *rel_dev) {
  if (!ctx) return RPA_ERR_ARG;
  if (!mesh || !G_occ || !G_un || ntau <= 0 || nb <= 0 || !(tol >= 0.0))
    return fail(ctx, RPA_ERR_ARG, "bad argument");
  for (int d = 0; d < 3; ++d)
    if (mesh[d] <= 0) return fail(ctx, RPA_ERR_ARG, "mesh must be positive");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  double *d = nullptr, h[2] = {0.0, 0.0};
  HIP_TRY(ctx, hipMalloc(&d, 2 * sizeof(double)));
  hipError_t e = launch_green_symmetry(G_occ, G_un, ntau, mesh, nb, d, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(ctx, RPA_ERR_HIP, std::string("symmetry check: ") + hipGetErrorString(e));
  const double rel = h[1] > 0.0 ? h[0] / h[1] : h[0];
  if (rel_dev) *rel_dev = rel;
  if (!(rel <= tol))
    return fail(ctx, RPA_ERR_ARG, "G(-R) differs from G(R)^T: relative deviation " + std::to_string(rel));
  return RPA_OK;
}

size_t rpa_ec_workspace_size(int n, int nq, int nomega) {
  if (n <= 0 || nq <= 0 || nomega <= 0) return 0;
  return ec_layout(n, nq, nomega, ec_default_batch(n, nq, nomega)).total;
}

int rpa_correlation_energy(rpa_ctx *ctx, int n, int nq, int nomega, const double *womega, const double *chi0_q,
                           const double *v_q, void *workspace, size_t workspace_bytes, double *Ec, double *Ec_q) {
  if (!ctx) return RPA_ERR_ARG;
  if (!womega || !chi0_q || !v_q || !workspace || !Ec) return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (n <= 0 || nq <= 0 || nomega <= 0) return fail(ctx, RPA_ERR_ARG, "sizes must be positive");
  EcLayout l;
  if (!ec_fit_layout(n, nq, nomega, workspace_bytes, l))
    return fail(ctx, RPA_ERR_WORKSPACE, "workspace smaller than rpa_ec_workspace_size with one matrix per batch");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  char *ws = (char *)workspace;
  double *wdev = (double *)(ws + l.w);
  HIP_TRY(ctx, hipMemcpyAsync(wdev, womega, nomega * 8, hipMemcpyHostToDevice, s));
  {
    Timed tm(ctx, "ec_stage");
    const int rc = ec_enqueue_known(ctx, s, n, nq, nomega, wdev, chi0_q, v_q, ws, l);
    if (rc != RPA_OK) return rc;
  }
  std::vector<int> hflags(nq + nq * nomega);
  std::vector<double> hecq(nq + 1);
  HIP_TRY(ctx, hipMemcpyAsync(hflags.data(), ws + l.flags, hflags.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(hecq.data(), ws + l.ecq, hecq.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  const int rc = ec_check_flags(ctx, hflags.data(), nq, nomega, "");
  if (rc != RPA_OK) return rc;
  *Ec = hecq[nq];
  if (Ec_q)
    for (int q = 0; q < nq; ++q) Ec_q[q] = hecq[q];
  return RPA_OK;
}

// ---- energy stage with the library's own device scratch (no allocation) ----
namespace {
// Every GPU the library runs on holds one copy of this array until the process ends.  In host
// code its name is only a stand-in: the device address comes from hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device; the device must be current.
hipError_t scratch_setup(int device, void **out) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!scratch_dev[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = p;
  }
  *out = scratch_dev[device];
  return hipSuccess;
}
}  // namespace

size_t rpa_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int rpa_correlation_energy_noalloc(rpa_ctx *ctx, int n, int nq, int nomega, const double *womega,
                                   const double *chi0_q, const double *v_q, double *Ec, double *Ec_q) {
  if (!ctx) return RPA_ERR_ARG;
  if (!womega || !chi0_q || !v_q || !Ec) return fail(ctx, RPA_ERR_ARG, "null pointer");
  if (n <= 0 || nq <= 0 || nomega <= 0) return fail(ctx, RPA_ERR_ARG, "sizes must be positive");
  // the scratch holds the energy-stage layout plus two status words at its end
  constexpr size_t kStatusBytes = 256;
  EcLayout l;
  if (!ec_fit_layout(n, nq, nomega, kNoAllocScratchBytes - kStatusBytes, l))
    return fail(ctx, RPA_ERR_WORKSPACE,
                "n = " + std::to_string(n) + ", nq = " + std::to_string(nq) +
                    " needs more than the 64 MiB device scratch of rpa_correlation_energy_noalloc");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  char *ws = (char *)ctx->scratch;
  if (!ws) return fail(ctx, RPA_ERR_HIP, "device scratch address was not set up for this context");
  hipStream_t s = ctx->stream;
  int *status = (int *)(ws + kNoAllocScratchBytes - kStatusBytes);
  double *wdev = (double *)(ws + l.w);
  HIP_TRY(ctx, hipMemcpyAsync(wdev, womega, nomega * 8, hipMemcpyHostToDevice, s));
  {
    Timed tm(ctx, "ec_stage");
    const int rc = ec_enqueue_known(ctx, s, n, nq, nomega, wdev, chi0_q, v_q, ws, l);
    if (rc != RPA_OK) return rc;
    HIP_TRY(ctx, launch_first_flag((const int *)(ws + l.flags), nq + nq * nomega, status, s));
  }
  int st[2] = {0, -1};
  const double *ecq = (const double *)(ws + l.ecq);
  HIP_TRY(ctx, hipMemcpyAsync(st, status, sizeof(st), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(Ec, ecq + nq, sizeof(double), hipMemcpyDeviceToHost, s));
  if (Ec_q) HIP_TRY(ctx, hipMemcpyAsync(Ec_q, ecq, (size_t)nq * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (st[0] != 0) {
    const int idx = st[1];
    if (idx < nq)
      return fail(ctx, RPA_ERR_NOT_HPD, "v(q) is not Hermitian positive definite at q index " + std::to_string(idx));
    const int q = (idx - nq) / nomega, k = (idx - nq) % nomega;
    if (st[0] == 1)
      return fail(ctx, RPA_ERR_NOT_HPD, "1 - L^H chi L is not positive definite at q index " + std::to_string(q) +
                                            ", omega index " + std::to_string(k));
    return fail(ctx, RPA_ERR_NONFINITE,
                "non-finite log-determinant at q index " + std::to_string(q) + ", omega index " + std::to_string(k));
  }
  return RPA_OK;
}

static void batch_release(rpa_batch *b) {
  if (!b) return;
  hipSetDevice(b->ctx->device);
  hipDeviceSynchronize();
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) hipEventDestroy(e);
  for (hipStream_t st : b->lanes) hipStreamDestroy(st);
  if (b->origin) hipStreamDestroy(b->origin);
  if (b->dparams) hipFree(b->dparams);
  if (b->dres) hipFree(b->dres);
  delete b;
}

// The whole path of one cell enqueued on stream s (the context's stream is pointed at s
// meanwhile); kernels only.
static int batch_enqueue_cell(rpa_batch *b, const BatchCell &c, hipStream_t s) {
  rpa_ctx *ctx = b->ctx;
  rpa_plan *p = c.io.plan;
  ctx->stream = s;
  char *bws = (char *)c.io.build_workspace;
  const double negs = -c.io.spin_factor;
  int rc = p->prec == RPA_FP64
               ? build_impl<double>(p, c.io.G_occ, c.io.G_un, c.io.C, bws, negs, c.io.chi0_tau, false)
               : build_impl<float>(p, c.io.G_occ, c.io.G_un, c.io.C, bws, negs, c.io.chi0_tau, p->prec == RPA_BF16X3);
  if (rc != RPA_OK) return rc;
  const size_t n2 = (size_t)c.n * c.n;
  HIP_TRY(ctx, launch_cos_transform(b->dparams + c.off_gamma, c.ntau, c.io.nomega, (size_t)c.nR * n2, c.io.chi0_tau,
                                    c.io.chi0_omega, s));
  HIP_TRY(ctx, launch_r2q(b->dparams + c.off_ph, c.nR, c.io.nq, c.io.nomega, n2, c.io.chi0_omega, c.io.chi0_q, s));
  char *ews = (char *)c.io.ec_workspace;
  rc = ec_enqueue(ctx, s, c.n, c.io.nq, c.io.nomega, b->dparams + c.off_w, c.io.chi0_q, c.io.v_q, ews, c.el);
  if (rc != RPA_OK) return rc;
  HIP_TRY(ctx, launch_copy_words(b->dres + c.off_flags, ews + c.el.flags, (size_t)c.io.nq * (1 + c.io.nomega), s));
  HIP_TRY(ctx, launch_copy_words(b->dres + c.off_ecq, ews + c.el.ecq, (size_t)2 * (c.io.nq + 1), s));
  return RPA_OK;
}

int rpa_batch_create(rpa_ctx *ctx, int ncells, int nlanes, const rpa_batch_cell *cells, rpa_batch **out) {
  if (!ctx) return RPA_ERR_ARG;
  if (!out || !cells) return fail(ctx, RPA_ERR_ARG, "null argument");
  *out = nullptr;
  if (ncells <= 0 || nlanes <= 0 || nlanes > 64) return fail(ctx, RPA_ERR_ARG, "need ncells > 0 and 1 <= nlanes <= 64");
  std::vector<BatchCell> bc(ncells);
  std::vector<double> params;
  size_t res = 0;
  auto pad = [&]() { params.resize((params.size() + 31) / 32 * 32, 0.0); };
  for (int i = 0; i < ncells; ++i) {
    const rpa_batch_cell &io = cells[i];
    const std::string at = "cell " + std::to_string(i) + ": ";
    if (!io.plan || io.plan->ctx != ctx) return fail(ctx, RPA_ERR_ARG, at + "plan missing or of another context");
    if (io.lane < 0 || io.lane >= nlanes) return fail(ctx, RPA_ERR_ARG, at + "lane out of range");
    if (!io.gamma_cos || !io.womega || !io.q_frac || !io.G_occ || !io.G_un || !io.v_q || !io.build_workspace ||
        !io.chi0_tau || !io.chi0_omega || !io.chi0_q || !io.ec_workspace || (io.plan->nblk > 0 && !io.C))
      return fail(ctx, RPA_ERR_ARG, at + "null pointer");
    if (io.nomega <= 0 || io.nomega > 64 || io.nq <= 0) return fail(ctx, RPA_ERR_ARG, at + "nomega in [1, 64], nq > 0");
    BatchCell &c = bc[i];
    c.io = io;
    c.n = io.plan->nauxtot;
    c.ntau = io.plan->ntau;
    c.nR = io.plan->nR;
    if ((size_t)2 * io.nq * c.nR * sizeof(double) > 64 * 1024)
      return fail(ctx, RPA_ERR_UNSUPPORTED, at + "nq * nR must not exceed 4096");
    if (io.build_workspace_bytes < io.plan->ws_total)
      return fail(ctx, RPA_ERR_WORKSPACE, at + "build workspace smaller than the plan's");
    if (!ec_fit_layout(c.n, io.nq, io.nomega, io.ec_workspace_bytes, c.el))
      return fail(ctx, RPA_ERR_WORKSPACE, at + "energy workspace too small");
    pad();
    c.off_gamma = params.size();
    params.insert(params.end(), io.gamma_cos, io.gamma_cos + (size_t)io.nomega * c.ntau);
    pad();
    c.off_ph = params.size();
    const std::vector<double> ph = r2q_phases(io.plan->mesh, io.nq, io.q_frac);
    params.insert(params.end(), ph.begin(), ph.end());
    pad();
    c.off_w = params.size();
    params.insert(params.end(), io.womega, io.womega + io.nomega);
    c.off_flags = res;
    res = align_up(res + (size_t)io.nq * (1 + io.nomega) * sizeof(int));
    c.off_ecq = res;
    res = align_up(res + (size_t)(io.nq + 1) * sizeof(double));
  }
  pad();
  rpa_batch *b = new rpa_batch();
  b->ctx = ctx;
  b->nlanes = nlanes;
  b->cells = bc;
  b->res_bytes = res;
  auto bail = [&](int code, const std::string &msg) {
    batch_release(b);
    return fail(ctx, code, msg);
  };
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMalloc(&b->dparams, params.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&b->dres, res);
  if (e == hipSuccess) e = hipMemcpy(b->dparams, params.data(), params.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->origin, hipStreamNonBlocking);
  for (int l = 0; l < nlanes && e == hipSuccess; ++l) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) b->lanes.push_back(st);
  }
  for (int k = 0; k <= nlanes && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->events.push_back(ev);
  }
  if (e != hipSuccess) return bail(RPA_ERR_HIP, std::string("batch setup: ") + hipGetErrorString(e));

  // capture: fork every lane off the origin stream, enqueue the cells, join
  e = hipStreamBeginCapture(b->origin, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return bail(RPA_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
  const hipStream_t saved_stream = ctx->stream;
  const bool saved_profile = ctx->profile;
  ctx->profile = false;
  int rc = RPA_OK;
  e = hipEventRecord(b->events[0], b->origin);
  for (int l = 0; l < nlanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], b->events[0], 0);
  if (e != hipSuccess) rc = fail(ctx, RPA_ERR_HIP, std::string("batch fork: ") + hipGetErrorString(e));
  for (int i = 0; i < ncells && rc == RPA_OK; ++i) {
    rc = batch_enqueue_cell(b, b->cells[i], b->lanes[b->cells[i].io.lane]);
    if (rc != RPA_OK) ctx->err = "cell " + std::to_string(i) + ": " + ctx->err;
  }
  ctx->stream = saved_stream;
  ctx->profile = saved_profile;
  for (int l = 0; l < nlanes && rc == RPA_OK; ++l) {
    e = hipEventRecord(b->events[1 + l], b->lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->origin, b->events[1 + l], 0);
    if (e != hipSuccess) rc = fail(ctx, RPA_ERR_HIP, std::string("batch join: ") + hipGetErrorString(e));
  }
  const hipError_t ee = hipStreamEndCapture(b->origin, &b->graph);
  if (rc != RPA_OK) {
    const std::string msg = ctx->err;
    batch_release(b);
    return fail(ctx, rc, msg);
  }
  if (ee != hipSuccess) return bail(RPA_ERR_HIP, std::string("end capture: ") + hipGetErrorString(ee));
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(RPA_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  *out = b;
  return RPA_OK;
}

int rpa_batch_run(rpa_batch *b) {
  if (!b) return RPA_ERR_ARG;
  rpa_ctx *ctx = b->ctx;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipGraphLaunch(b->exec, ctx->stream));
  return RPA_OK;
}

int rpa_batch_result(rpa_batch *b, double *Ec, double *Ec_q) {
  if (!b) return RPA_ERR_ARG;
  rpa_ctx *ctx = b->ctx;
  if (!Ec) return fail(ctx, RPA_ERR_ARG, "null pointer");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  std::vector<char> h(b->res_bytes);
  HIP_TRY(ctx, hipMemcpyAsync(h.data(), b->dres, b->res_bytes, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  size_t qo = 0;
  for (size_t i = 0; i < b->cells.size(); ++i) {
    const BatchCell &c = b->cells[i];
    const int rc = ec_check_flags(ctx, (const int *)(h.data() + c.off_flags), c.io.nq, c.io.nomega,
                                  "cell " + std::to_string(i) + ": ");
    if (rc != RPA_OK) return rc;
    const double *ecq = (const double *)(h.data() + c.off_ecq);
    Ec[i] = ecq[c.io.nq];
    if (Ec_q)
      for (int q = 0; q < c.io.nq; ++q) Ec_q[qo + q] = ecq[q];
    qo += c.io.nq;
  }
  return RPA_OK;
}

int rpa_batch_destroy(rpa_batch *b) {
  if (!b) return RPA_ERR_ARG;
  batch_release(b);
  return RPA_OK;
}

#ifdef RPA_HOST_TABLE_TEST
// Entry points of the host-only table build: a context without a device, and a summary of a
// plan's tables for the sanitizer test's consistency checks.
rpa_ctx *rpa_test_host_ctx(void) { return new rpa_ctx(); }
void rpa_test_host_ctx_free(rpa_ctx *ctx) { delete ctx; }
int rpa_test_plan_summary(const rpa_plan *p, long long *out) {
  if (!p || !out) return RPA_ERR_ARG;
  long long sl = 0;
  for (int a = 0; a < p->natoms; ++a) sl += p->nslices[a];
  out[0] = (long long)p->ws_total;
  out[1] = (long long)p->itemU.size();
  out[2] = (long long)p->tileV.size();
  out[3] = (long long)p->groups.size();
  out[4] = p->n_elems;
  out[5] = p->ns_elems;
  out[6] = sl;
  out[7] = (long long)p->half_order.size();
  return RPA_OK;
}
#endif

}  // extern "C"
