/*
 * rpa_mi355x.h - C ABI of the MI355X (gfx950) library for the space-time
 * chi0 -> RPA correlation energy path of the LRI/NAO low-scaling RPA method
 * (arXiv 2407.19930, Sec. 2 and Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Plain pointers and sizes only.  "device" arrays live in GPU memory owned
 *   by the caller (for instance torch tensors' data_ptr()); "host" arrays live
 *   in CPU memory owned by the caller.  The library never frees or keeps a
 *   caller pointer beyond the call.
 * - Row-major, contiguous.  Complex numbers are interleaved (re, im) FP64.
 * - All device work of a call is queued on the context's HIP stream and is
 *   asynchronous with respect to the host, except where a call returns host
 *   values (rpa_correlation_energy), which synchronises the stream.
 * - Real-valued convention for tau > 0 (Sec. 2, Eq. (green_mat)): the paper's
 *   G(R, i tau) = i G^un(R, tau) and G(R, -i tau) = -i G^occ(R, tau) with
 *   G^occ, G^un real; the paper's chi0(R, i tau) = i chi(R, tau) with chi real.
 *   The inputs must satisfy G^s(-R) = G^s(R)^T (real Hermitian Green's
 *   functions, time-reversal symmetric); the kernels rely on it.
 * - BvK supercell: lattice vectors R are integer triples n in
 *   [0,N1)x[0,N2)x[0,N3) flattened as (n1*N2 + n2)*N3 + n3; the k/q mesh
 *   (Gamma-centred, k = n/N) uses the same ordering.
 * - Return value: RPA_OK (0) or an rpa_status error code; nothing is thrown
 *   across the ABI.  rpa_last_error() returns a message for the last failing
 *   call on a context.  On error, output arrays are unspecified and inputs are
 *   unchanged (inputs are never written).
 */
#ifndef RPA_MI355X_H
#define RPA_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define RPA_API __attribute__((visibility("default")))
#else
#define RPA_API
#endif

typedef enum {
  RPA_OK = 0,
  RPA_ERR_ARG = 1,          /* null pointer, bad enum, negative size */
  RPA_ERR_SHAPE = 2,        /* inconsistent sizes (atoms, blocks, mesh, tau) */
  RPA_ERR_WORKSPACE = 3,    /* workspace smaller than the queried size */
  RPA_ERR_NOT_HPD = 4,      /* a matrix to be Cholesky-factorised is not Hermitian positive definite */
  RPA_ERR_NONFINITE = 5,    /* NaN or Inf met in a reduction */
  RPA_ERR_HIP = 6,          /* HIP runtime error */
  RPA_ERR_UNSUPPORTED = 7   /* shape outside the compiled kernel limits */
} rpa_status;

/* Arithmetic of the chi0 build.  G is always passed in FP64; the FP32 and BF16X3
 * paths scale G^occ and G^un of each tau by powers of two (max abs in [1, 2)) before
 * the cast and remove the scale in FP64 when writing chi. */
typedef enum {
  RPA_FP64 = 0,             /* every contraction in FP64 (MFMA f64) */
  RPA_FP32 = 1,             /* contractions in FP32 (MFMA f32), FP64 across neighbour blocks */
  RPA_BF16X3 = 2            /* the N stage and the neighbour loop (O and chi += C O) in split
                               BF16: x = hi + lo, a b = a_hi b_hi + a_hi b_lo + a_lo b_hi on the
                               bf16 MFMAs, FP32 accumulation, FP64 across neighbour blocks; the
                               Z terms in FP32.  A plan whose split operands of the N stage
                               exceed 4 GiB per part runs that stage as RPA_FP32 */
} rpa_precision;

typedef struct rpa_ctx rpa_ctx;
typedef struct rpa_plan rpa_plan;

/* One periodic cell: atoms with their NAO / ABF counts and the k-mesh (= BvK
 * supercell).  Limits of this build: nao[a] <= 32, naux[a] <= 128. */
typedef struct {
  int natoms;
  const int *nao;           /* host [natoms] */
  const int *naux;          /* host [natoms] */
  int mesh[3];              /* N1, N2, N3 >= 1 */
} rpa_cell;

/* LRI triple coefficients (Sec. 2, Eq. (eq:LRI)): one block per ordered
 * neighbour pair (I, K(R)) with the ABF index on I, stored as
 * C[off[b] + (mu * nao[I] + i) * nao[K] + k] = C^{mu(0)}_{i(0), k(R)}.
 * The set of blocks with first atom U is the neighbourhood N[U] of
 * Algorithm 1.  Blocks are read, never written; their order is free. */
typedef struct {
  int nblk;
  const int *I;             /* host [nblk] */
  const int *K;             /* host [nblk] */
  const int *R;             /* host [3*nblk], unfolded integer lattice vector of K */
  const long long *off;     /* host [nblk], element offset of the block in C */
} rpa_lri_blocks;

/* Create / destroy a context bound to one device and one HIP stream
 * (hip_stream may be NULL for the default stream; pass torch's current stream
 * to order the library's work with torch's). */
RPA_API int rpa_create(rpa_ctx **ctx, int device, void *hip_stream);
RPA_API int rpa_set_stream(rpa_ctx *ctx, void *hip_stream);
RPA_API void rpa_destroy(rpa_ctx *ctx);
RPA_API const char *rpa_last_error(const rpa_ctx *ctx);

/* Plan for one cell: neighbour tables, BvK fold tables and work lists of
 * Algorithm 1 (atom pairs U <= V, Sec. 3.2; lattice vectors R; tau points).
 * The plan owns small device tables; *workspace_bytes receives the size of the
 * caller-owned device workspace every compute call of this plan needs.  A plan
 * must be destroyed before its context; rpa_plan_destroy waits for the device.
 * Errors: RPA_ERR_ARG, RPA_ERR_SHAPE, RPA_ERR_UNSUPPORTED, RPA_ERR_HIP. */
RPA_API int rpa_plan_create(rpa_ctx *ctx, const rpa_cell *cell, const rpa_lri_blocks *blocks,
                    int ntau, int precision, size_t *workspace_bytes, rpa_plan **plan);
RPA_API int rpa_plan_destroy(rpa_plan *plan);

/* Algorithmic flop count of the chi0 build for this plan (Algorithm 1 with
 * its N intermediate evaluated once per (V, K, R1-R)), and the flops the
 * kernels actually execute (padding excluded). Host values. */
RPA_API int rpa_plan_flops(const rpa_plan *plan, double *alg_flops, double *exec_flops);

/* Per-kernel split of the same counts: stage 0 = N-stage kernel (the N intermediate
 * of Algorithm 1), stage 1 = fused kernel (X, M, Z, O and chi += C O of Algorithm 1).
 * Errors: RPA_ERR_ARG. */
RPA_API int rpa_plan_stage_flops(const rpa_plan *plan, int stage, double *alg_flops, double *exec_flops);

/* Launch variants of a plan's two chi0 kernels (the tunable part of the batched
 * build: how the uneven atom-pair work lists are laid over the chip's XCDs, and
 * the K step of the N-stage GEMM).  Workgroups are dealt to the 8 XCDs (each with
 * its own L2) round-robin; in the XCD-grouped order each XCD runs one contiguous
 * range of the plan-order list, so neighbouring tiles or items share its L2.
 *   nstage_order : 0 plan order, 1 XCD-grouped (N-stage tiles)
 *   nstage_kstep : 16 or 32 for the FP32 and FP64 N-stage kernel; 0 where the
 *                  plan's N stage has no such choice (the split-BF16 N stage)
 *   fused_order  : 0 plan order, 1 XCD-grouped (fused-kernel items)
 *   from_cache   : 1 if rpa_plan_autotune took the choice from the context's cache
 *   nstage_ms, fused_ms : measured duration of one tau with the chosen variants
 *                  (0 when not measured)
 *   fused_single : 0 one fused launch per template class (the atom classes of the
 *                  uneven blocks: ABF tiles of U, NAO steps of V, NAO tiles of U) and tau;
 *                  1, 2 or 3 (split-BF16 plans only) one launch for every class and every tau
 *                  of a chunk (rpa_plan_set_tau_batch), with the work of each tau in order of
 *                  decreasing size so that the compute units that finish early take the
 *                  small items; 1: workgroups of 8 waves, one per item (up to 128 ABF columns
 *                  of V); 2: workgroups of 4 waves, one per half of an item's columns (an
 *                  item with at most 64 columns takes one), two workgroups per compute unit;
 *                  3: workgroups of 4 waves, one per item, each wave two tiles of 16 columns
 *                  (one wave per SIMD; each C fragment read feeds both tiles)
 *   nstage_bm    : rows of an N-stage output tile: 128 (4 waves), or 256 (8 waves, each
 *                  staged C tile used for twice the rows; split-BF16 N stage only)
 * Every variant computes the same chi; the item order leaves it bitwise unchanged,
 * the K step changes the FP32/FP64 summation order only. */
typedef struct {
  int nstage_order;
  int nstage_kstep;
  int fused_order;
  int from_cache;
  double nstage_ms;
  double fused_ms;
  int fused_single;
  int nstage_bm;
} rpa_tuning;

/* Autotuner: times every variant of the N-stage kernel, then of the fused kernel,
 * on the first tau of the given inputs (one warm-up and one timed launch each, HIP
 * events on the context's stream), keeps the fastest in the plan (the defaults unless
 * another variant is at least 2% faster) and caches it in
 * the context under the plan's shape class (precision, atom and basis counts,
 * lattice-vector count, LRI block count, work-list sizes) and the device's
 * architecture name; a later plan of the same class takes the cached choice
 * without timing.  Inputs as for build_chi0_tau; chi0_scratch is a device FP64
 * buffer of nR * naux_tot^2 elements that receives chi of the first tau.  Blocks
 * the host until the timing is done.  *out (host, may be null) receives the choice.
 * Errors: RPA_ERR_ARG, RPA_ERR_WORKSPACE, RPA_ERR_HIP. */
RPA_API int rpa_plan_autotune(rpa_plan *plan, double spin_factor, const double *G_occ, const double *G_un,
                              const double *C, void *workspace, size_t workspace_bytes, double *chi0_scratch,
                              rpa_tuning *out);
/* The plan's current variants (defaults: plan orders, K step 16 (0 on the split-BF16 N stage),
 * per-class fused launches, N-stage tiles of 128 rows).  Errors: RPA_ERR_ARG. */
RPA_API int rpa_plan_get_tuning(const rpa_plan *plan, rpa_tuning *out);
/* Sets the variants explicitly (from_cache and the times are ignored); values outside
 * the ranges above are rejected with RPA_ERR_ARG and leave the plan unchanged. */
RPA_API int rpa_plan_set_tuning(rpa_plan *plan, const rpa_tuning *t);

/* tau points per launch.  By default every tau runs its own N-stage and fused launches (the
 * workspace holds padded G and the N intermediate of one tau).  rpa_plan_set_tau_batch sets
 * ntau_per_launch in [1, ntau]: G of that many tau points is padded and screened in turn, then one
 * N-stage launch and one fused launch (or one per template class and tau, see fused_single) cover
 * them all, and the workspace holds their padded G and N side by side.  *workspace_bytes receives
 * the new workspace size (for the N intermediate it grows with ntau_per_launch); every later
 * compute call of the plan needs that much.  rpa_plan_workspace_bytes returns the current size.
 * Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int rpa_plan_set_tau_batch(rpa_plan *plan, int ntau_per_launch, size_t *workspace_bytes);
RPA_API int rpa_plan_workspace_bytes(const rpa_plan *plan, size_t *workspace_bytes);

/* Green's-function screening of the chi0 build (the paper's lever for linear scaling: the
 * decay of G limits the range of the lattice vector R on top of the locality of the LRI
 * neighbourhoods, Sec. 2 after Algorithm 1; its case study screens on G with a threshold of
 * 1e-3, Sec. 6).  The paper states no rule; this library bounds every term of Algorithm 1 by its
 * two Green's-function factors.  Per tau, from the FP64 G input:
 *   gb(U, V, R)  = max over s, i in U, j in V of |G^s_ij(R, tau)|
 *   gn(V, K, dR) = max over L(dL) in N[V] of gb(L, K, dR - dL)   (bounds every G inside N(V, K, dR))
 *   g            = max of gb,  cut = (theta g) g
 * For the block chi_UV(R, tau), the M terms of neighbour K(R1) of U (G_UV(R) times N(V, K, R1 - R))
 * are dropped when gb(U, V, R) gn(V, K, R1 - R) < cut, and the Z terms when
 * gn(U, V, R) gn(V, U, -R) < cut (FP64 products; a block whose terms are all dropped is written as
 * zero, which restricts the R range).  theta = 0 (the default) drops nothing and gives exactly the
 * unscreened build; theta > 1 drops everything.  Every dropped term is bounded elementwise by
 * 2 s gb gn times sums of |C|, so the error vanishes with theta.
 * rpa_plan_set_screening sets theta (finite, >= 0; RPA_ERR_ARG otherwise) for the following
 * builds of the plan, and on first use with theta > 0 allocates a small plan-owned device buffer
 * (2 natoms^2 nR doubles of bounds and 3 ints per fused-kernel item and tau of statistics).
 * rpa_plan_screening_stats waits for the context's stream and returns, for the last
 * build_chi0_tau of the plan with screening on (RPA_ERR_ARG if there is none since theta was
 * set), host out[6] = {neighbour entries kept, entries in total, K(R1) slices kept, slices in
 * total, blocks whose Z terms were kept, blocks in total}, summed over all (U <= V, R, tau).
 * Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int rpa_plan_set_screening(rpa_plan *plan, double theta);
RPA_API int rpa_plan_screening_stats(rpa_plan *plan, long long *out);

/* Opt-in kernel timing with HIP events recorded on the context's stream around
 * every launch of the library's kernels.  rpa_profile(ctx, 1) enables and resets,
 * rpa_profile(ctx, 0) disables.  rpa_profile_read waits for the recorded events and
 * returns the summed duration and launch count of one kernel ("pack_c", "pad_g",
 * "screen", "nstage", "split_n", "fused", "cos_transform", "r2q", "ec_stage", "green").  Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int rpa_profile(rpa_ctx *ctx, int enable);
RPA_API int rpa_profile_read(rpa_ctx *ctx, const char *kernel, double *total_ms, int *launches);

/* chi(R, tau) of Algorithm 1 for every atom pair and lattice vector
 * (Sec. 2, the chi0_{mu,nu}(R, i tau) formula; Algorithm 1):
 *   chi_{mu nu}(R, tau) = -s sum_{K(R1) in N[U]} sum_{i k} C^mu_{ik}(R1) O^nu_{ik}(R1, R, tau) + ...
 * with s = spin_factor (2 for closed shells).
 *   G_occ, G_un : device FP64 [ntau][nR][nb][nb]  (nb = sum of nao)
 *   C           : device FP64, blocks as described by rpa_lri_blocks
 *   workspace   : device, at least the size returned by rpa_plan_create
 *   chi0_tau    : device FP64 [ntau][nR][naux_tot][naux_tot], written in full
 * Errors: RPA_ERR_ARG, RPA_ERR_WORKSPACE, RPA_ERR_HIP. */
RPA_API int build_chi0_tau(rpa_plan *plan, double spin_factor, const double *G_occ, const double *G_un,
                   const double *C, void *workspace, size_t workspace_bytes, double *chi0_tau);

/* Green's functions of the chi0 build from Bloch eigenpairs (Sec. 2, Eq. (green_mat), the
 * factors of i taken out: for tau > 0 the paper's G(R, i tau) = i G^un(R, tau) and
 * G(R, -i tau) = -i G^occ(R, tau)):
 *   G^occ_{ij}(R, tau) = (1/N_k) sum_k e^{-i k.R} sum_{n < nocc}  c_{in}(k) c*_{jn}(k) e^{-(mu - eps_nk) tau}
 *   G^un_{ij}(R, tau)  = (1/N_k) sum_k e^{-i k.R} sum_{n >= nocc} c_{in}(k) c*_{jn}(k) e^{-(eps_nk - mu) tau}
 * on the BvK lattice vectors of mesh (flattened index n1 N2 N3 + n2 N3 + n3, the order of chi's
 * R axis), k.R = 2 pi k_frac . n_R.
 *   tau         : host FP64 [ntau]          k_frac : host FP64 [nk][3]
 *   eps         : device FP64 [nk][nb], band energies; the first nocc bands are occupied at every k
 *   wfc         : device complex128 [nk][nb][nb], c_{in}(k) at [k][i][n] (eigenvectors in columns)
 *   workspace   : device, at least rpa_green_workspace_size(nk, nb, nocc) bytes
 *   G_occ, G_un : device FP64 [ntau][nR][nb][nb], written in full: the real part (the imaginary
 *                 part vanishes when H(-k) = H(k)*, as for the real hoppings of the path)
 * The output is the G_occ / G_un input of build_chi0_tau.  Asynchronous on the context's stream.
 * Errors: RPA_ERR_ARG, RPA_ERR_UNSUPPORTED (nR * nk > 4096), RPA_ERR_WORKSPACE, RPA_ERR_HIP. */
RPA_API size_t rpa_green_workspace_size(int nk, int nb, int nocc);
RPA_API int build_green_tau(rpa_ctx *ctx, int nk, int nb, int nocc, double mu, int ntau, const double *tau,
                            const int mesh[3], const double *k_frac, const double *eps, const double *wfc,
                            void *workspace, size_t workspace_bytes, double *G_occ, double *G_un);

/* Check of the precondition of build_chi0_tau that the Green's functions are real and symmetric
 * under R -> -R with transposition, G^s(-R) = G^s(R)^T (time reversal; the kernels take the X
 * intermediate of Algorithm 1 as a transposed N block and rely on it):
 *   G_occ, G_un : device FP64 [ntau][nR][nb][nb] on the BvK mesh `mesh`
 *   *rel_dev    : host, receives max |G^s(-R)_ji - G^s(R)_ij| / max |G^s(R)_ij| (may be null)
 * Returns RPA_ERR_ARG when the relative deviation exceeds tol (or is not a number); inputs that
 * fail it give a chi that is not Algorithm 1's.  Synchronises the context's stream.
 * Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int rpa_check_green_symmetry(rpa_ctx *ctx, int ntau, const int mesh[3], int nb, const double *G_occ,
                                     const double *G_un, double tol, double *rel_dev);

/* Cosine transform tau -> i omega (Sec. 2, the chi0(R, i omega_k) equation):
 *   chi(R, i omega_k) = sum_j Gamma_kj chi(R, tau_j),  Gamma_kj = gamma_jk cos(tau_j omega_k)
 * (the paper's -i and chi0 = i chi cancel).
 *   gamma_cos  : host FP64 [nomega][ntau]
 *   chi0_tau   : device FP64 [ntau][n]   chi0_omega : device FP64 [nomega][n]
 *   n          : elements per time point (nR * naux_tot^2 for a plan's chi)
 * Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int chi0_tau_to_omega(rpa_ctx *ctx, int ntau, int nomega, size_t n, const double *gamma_cos,
                      const double *chi0_tau, double *chi0_omega);

/* Fourier transform R -> q (Sec. 2, the chi0(q, i omega) equation):
 *   chi(q) = sum_R exp(2 pi i q_frac . n_R) chi(R)
 *   mesh        : BvK mesh of the R axis (nR = N1 N2 N3)
 *   q_frac      : host FP64 [nq][3] fractional reciprocal coordinates
 *   chi0_R      : device FP64 [nbatch][nR][m]
 *   chi0_q      : device complex128 interleaved [nbatch][nq][m]
 * Errors: RPA_ERR_ARG, RPA_ERR_HIP. */
RPA_API int chi0_R_to_q(rpa_ctx *ctx, const int mesh[3], int nbatch, size_t m, int nq, const double *q_frac,
                const double *chi0_R, double *chi0_q);

/* Correlation energy (Sec. 2, the E_c^RPA equations with Tr ln = ln det):
 *   E_c = 1/(2 pi) 1/nq sum_q sum_k w_k { ln det[1 - chi(q, i w_k) v(q)] + Tr[chi v] }
 * evaluated as ln det(I - B) + Tr B with B = L^H chi L, v(q) = L L^H (Cholesky,
 * FP64), det(1 - chi L L^H) = det(I - L^H chi L); I - B is Hermitian positive
 * definite when chi is negative semidefinite, and its log-determinant is
 * twice the sum of the logs of its Cholesky diagonal.  A q point whose
 * chi(q, i w_k) (every k) has zero imaginary parts takes T = chi L with two real
 * products per complex one; where v(q) is real as well (a time-reversal
 * invariant q with a real basis) every step of that q runs on real matrices.
 * The choice is made on the device per q, so one call may mix both kinds.
 *   n           : matrix order (naux_tot)
 *   womega      : host FP64 [nomega]
 *   chi0_q      : device complex128 [nomega][nq][n][n]
 *   v_q         : device complex128 [nq][n][n], Hermitian positive definite
 *   workspace   : device; rpa_ec_workspace_size(n, nq, nomega) bytes run the
 *                 (q, omega) pairs in batches of up to all nq * nomega of them
 *                 (at most 64 GiB of per-pair matrices); less, down to the size
 *                 for one pair per batch, runs smaller batches
 *   Ec          : host, E_c per cell (Hartree)
 *   Ec_q        : host [nq] per-q contributions (already divided by nq), or NULL
 * Synchronises the stream.  Errors: RPA_ERR_ARG, RPA_ERR_WORKSPACE,
 * RPA_ERR_NOT_HPD (v(q) or I - B not HPD; the message names q and omega index),
 * RPA_ERR_NONFINITE, RPA_ERR_HIP. */
RPA_API size_t rpa_ec_workspace_size(int n, int nq, int nomega);
RPA_API int rpa_correlation_energy(rpa_ctx *ctx, int n, int nq, int nomega, const double *womega,
                           const double *chi0_q, const double *v_q, void *workspace,
                           size_t workspace_bytes, double *Ec, double *Ec_q);

/* Energy stage without device allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same result
 * as rpa_correlation_energy (same kernels, same order), with its workspace taken from a device
 * array of rpa_noalloc_scratch_bytes() = 64 MiB that the library holds on every GPU it runs on
 * until the process ends.  No hipMalloc, hipFree or other allocation happens in the call.
 *   n, nq, nomega, womega, chi0_q, v_q, Ec, Ec_q : as rpa_correlation_energy
 * Sizes whose energy-stage workspace (with one (q, omega) matrix per batch) exceeds the scratch
 * are rejected with RPA_ERR_WORKSPACE.  Every call on one GPU shares that GPU's scratch and
 * leaves its contents behind; calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller.  Synchronises the context's stream.
 * Errors: RPA_ERR_ARG, RPA_ERR_WORKSPACE, RPA_ERR_NOT_HPD, RPA_ERR_NONFINITE, RPA_ERR_HIP. */
RPA_API size_t rpa_noalloc_scratch_bytes(void);
RPA_API int rpa_correlation_energy_noalloc(rpa_ctx *ctx, int n, int nq, int nomega, const double *womega,
                                           const double *chi0_q, const double *v_q, double *Ec, double *Ec_q);

/* ---- Batches of independent cells -------------------------------------------
 * The whole path (build_chi0_tau, chi0_tau_to_omega, chi0_R_to_q and the energy
 * stage of rpa_correlation_energy) of many cells, captured once into one HIP graph
 * and replayed with a single graph launch.  Cells are assigned to lanes: the cells
 * of a lane run one after another in the order given, lanes run concurrently
 * (one stream branch per lane inside the graph).  Cells of one lane may therefore
 * share scratch buffers (chi arrays, workspaces); cells of different lanes must not.
 * Small per-cell host arrays are copied at creation; device pointers are captured
 * into the graph and must stay valid, with the same sizes, while the batch lives. */
typedef struct rpa_batch rpa_batch;

typedef struct {
  rpa_plan *plan;           /* the cell's plan (cell shape, ntau, precision); same context */
  int lane;                 /* 0 <= lane < nlanes */
  int nomega, nq;
  double spin_factor;
  const double *gamma_cos;  /* host [nomega][ntau], as chi0_tau_to_omega */
  const double *womega;     /* host [nomega] */
  const double *q_frac;     /* host [3*nq] */
  const double *G_occ, *G_un, *C;   /* device, as build_chi0_tau */
  const double *v_q;        /* device complex128 [nq][n][n] (n = the cell's naux total) */
  void *build_workspace;    /* device, >= the plan's workspace size */
  size_t build_workspace_bytes;
  double *chi0_tau;         /* device [ntau][nR][n][n] */
  double *chi0_omega;       /* device [nomega][nR][n][n] */
  double *chi0_q;           /* device complex128 [nomega][nq][n][n]; may alias chi0_tau when
                               that buffer holds 2 nomega nR n^2 doubles (chi0_tau is dead
                               once chi0_omega is built) */
  void *ec_workspace;       /* device, >= rpa_ec_workspace_size(n, nq, nomega) with one
                               frequency per batch (see rpa_correlation_energy) */
  size_t ec_workspace_bytes;
} rpa_batch_cell;

/* Validate the cells, copy their host arrays to the device and capture the graph
 * (nothing runs yet).  Errors: RPA_ERR_ARG, RPA_ERR_SHAPE, RPA_ERR_WORKSPACE,
 * RPA_ERR_HIP. */
RPA_API int rpa_batch_create(rpa_ctx *ctx, int ncells, int nlanes, const rpa_batch_cell *cells,
                             rpa_batch **batch);
/* Launch the graph on the context's stream (asynchronous). */
RPA_API int rpa_batch_run(rpa_batch *batch);
/* Wait for the stream, check every cell's status flags and copy E_c per cell
 * (host [ncells]) and, if Ec_q is not NULL, the per-q terms of all cells
 * concatenated in cell order (host [sum of nq]).  Errors: RPA_ERR_NOT_HPD,
 * RPA_ERR_NONFINITE (the message names the cell), RPA_ERR_HIP. */
RPA_API int rpa_batch_result(rpa_batch *batch, double *Ec, double *Ec_q);
/* Waits for the device, then frees the graph, the lane streams and the batch's
 * small device buffers.  The plans stay owned by the caller. */
RPA_API int rpa_batch_destroy(rpa_batch *batch);

/* ---- Input session shaped like the paper's library interface (App. B) -----------------
 * For host programs (NAO DFT codes) that hand over their data the way the paper's interface
 * takes it: dimensions, band energies and occupations, Bloch eigenvectors per k, lattice and k
 * mesh, irreducible k points with weights, LRI coefficients per atom pair with a lattice vector,
 * the Coulomb matrix per atom pair or per 2D block, then one call for the correlation energy.
 * All arrays are HOST arrays owned by the caller and copied by the call; the session keeps its
 * own host copies, and rpa_get_rpa_correlation_energy allocates and frees the device memory it
 * needs.  Units: Hartree and Bohr (or any consistent pair).  Closed shells only.
 * Readings of the listing: rpa_corr and rpa_corr_irk_contrib are real (E_c is real by
 * construction); wfc_real / wfc_imag hold c_{i n}(k) band-major, [nstates][nbasis]; wg are
 * occupation weights, and a band counts as occupied when |wg| exceeds half the largest |wg| (the
 * occupied bands must come first and be as many at every k: an insulator); the minimax time and
 * frequency grids, which the paper's library generates itself, are an input here
 * (rpa_set_time_freq_grids).  Errors: RPA_ERR_ARG, RPA_ERR_SHAPE, RPA_ERR_UNSUPPORTED and those
 * of the compute calls; rpa_session_last_error() describes the last one. */
typedef struct rpa_session rpa_session;
RPA_API int rpa_session_create(rpa_ctx *ctx, rpa_session **session);
RPA_API int rpa_session_destroy(rpa_session *session);
RPA_API const char *rpa_session_last_error(const rpa_session *session);
/* Arithmetic of the chi0 build (rpa_precision; RPA_FP64 by default). */
RPA_API int rpa_session_set_precision(rpa_session *session, int precision);
/* nspins (must be 1), nkpts (= N1 N2 N3 of the k mesh), nstates (bands), nbasis (NAOs of the
 * cell), natoms.  Resets the eigenvectors and bands. */
RPA_API int rpa_set_dimension(rpa_session *session, int nspins, int nkpts, int nstates, int nbasis, int natoms);
/* wg, ekb: [nspins][nkpts][nstates] occupation weights and band energies; efermi: the chemical
 * potential mu of the Green's functions. */
RPA_API int rpa_set_wg_ekb_efermi(rpa_session *session, int nspins, int nkpts, int nstates, const double *wg,
                                  const double *ekb, double efermi);
/* Eigenvectors at (ispin, ik): wfc_real, wfc_imag [nstates][nbasis], c_{i n}(k) at [n][i]. */
RPA_API int rpa_set_ao_basis_wfc(rpa_session *session, int ispin, int ik, const double *wfc_real,
                                 const double *wfc_imag);
/* lat_mat: lattice vectors a_d as rows; G_mat: reciprocal vectors as rows (kept, not needed). */
RPA_API int rpa_set_latvec_and_G(rpa_session *session, const double lat_mat[9], const double G_mat[9]);
/* k mesh N1 x N2 x N3 (Gamma-centred BvK mesh) and the Cartesian k vectors [nkpts][3] in the
 * mesh order (k index (n1 N2 + n2) N3 + n3); fractional coordinates are k . a_d / (2 pi). */
RPA_API int rpa_set_kgrids_kvec_tot(rpa_session *session, int nk1, int nk2, int nk3, const double *kvecs);
/* Irreducible k (= q) points: indices into the k list and weights (normalised to sum 1 by the
 * library).  Without this call every k point is a q point of weight 1/nkpts.  Clears the Coulomb
 * matrices set so far (their q index refers to this list). */
RPA_API int rpa_set_ibz2bz_index_and_weight(rpa_session *session, int nk_irk, const int *ibz2bz_index,
                                            const double *wk_irk);
/* LRI block of atom I with atom J displaced by the integer lattice vector R[3]:
 * Cs_in[mu][i][j] for mu on I (naux_mu), i on I (nbasis_i), j on J (nbasis_j), as rpa_lri_blocks;
 * insert_index_only = 1 registers the block with zero coefficients.  A later call for the same
 * (I, J, R) replaces the block.  Every atom needs its own block (I, I, 0) for its sizes. */
RPA_API int rpa_set_ao_basis_aux(rpa_session *session, int I, int J, int nbasis_i, int nbasis_j, int naux_mu,
                                 const int *R, const double *Cs_in, int insert_index_only);
/* Coulomb matrix v(q) of q index ik (into the irreducible list, or the k list): the block of atoms
 * (I, J), [naux_mu][naux_nu] real and imaginary parts (needs the LRI blocks for the ABF offsets),
 * or the block [mu_begin, mu_end) x [nu_begin, nu_end) of the max_naux x max_naux matrix.  Every
 * element of every q must be set before the energy call. */
RPA_API int rpa_set_aux_bare_coulomb_k_atom_pair(rpa_session *session, int ik, int I, int J, int naux_mu,
                                                 int naux_nu, const double *Vq_real_in, const double *Vq_imag_in);
RPA_API int rpa_set_aux_bare_coulomb_k_2D_block(rpa_session *session, int ik, int max_naux, int mu_begin,
                                                int mu_end, int nu_begin, int nu_end, const double *Vq_real_in,
                                                const double *Vq_imag_in);
/* Minimax grids: tau[ngrid], frequency weights[ngrid] and the cosine-transform weights
 * gamma_cos[ngrid][ngrid] (as chi0_tau_to_omega) with as many frequencies as time points. */
RPA_API int rpa_set_time_freq_grids(rpa_session *session, int ngrid, const double *tau, const double *omega_weights,
                                    const double *gamma_cos);
/* Runs build_green_tau, build_chi0_tau, chi0_tau_to_omega, chi0_R_to_q and rpa_correlation_energy on
 * the session's data (the q points of the irreducible list) and returns *rpa_corr = E_c per cell
 * and, if rpa_corr_irk_contrib is not null, the contribution of every irreducible q point,
 * w_q (1/2 pi) sum_k w_k {ln det[1 - chi0 v] + Tr[chi0 v]} ([nk_irk], summing to E_c). */
RPA_API int rpa_get_rpa_correlation_energy(rpa_session *session, double *rpa_corr, double *rpa_corr_irk_contrib);

#ifdef __cplusplus
}
#endif

#endif /* RPA_MI355X_H */
