/*
 * amg.h - C ABI of libamg, an MI355X (gfx950) adaptive multigrid solver for
 * the Wilson-Dirac equation D(U) psi = chi (Eq. (1) of Brannick, Brower,
 * Clark, Osborn, Rebbi, "Adaptive Multigrid Algorithm for Lattice QCD",
 * arXiv:0707.4018).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named dev_* are HIP device pointers; everything else is host.
 *   `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *   on `stream` and may still be running when a call returns, except where a
 *   call documents a host synchronisation.
 * - Canonical field layout (all dev_* fields crossing the ABI): complex
 *   numbers interleaved (re, im), lexicographic sites with x_1 fastest, then
 *   spin, then colour:  psi[rhs][site][spin][colour].  Complex128 unless an
 *   entry point takes an amg_prec argument.  Two dimensions: n_s = 2,
 *   n_c = 1 (U(1)); four dimensions: n_s = 4, n_c = 3 (SU(3)).
 * - Canonical gauge layout: U[mu][site][a][b] complex128, row-major colour,
 *   mu = 0..nd-1 the direction of x_{mu+1}.
 * - Gamma matrices: 2d gamma_1 = sigma_1, gamma_2 = sigma_2; 4d chiral basis
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]];
 *   gamma_5 is diagonal, +1 on the first half of the spin components.
 * - Coarse fields (levels >= 1) are psi[rhs][coarse site][t], t = chi*N_v + k
 *   (chirality major), complex128.
 * - Ownership: the caller owns every dev_* buffer and must keep inputs alive
 *   until `stream` has passed the call.  Handles own their internal device
 *   memory (hipMalloc, or the routines given to amg_set_allocator) and free
 *   it in amg_*_destroy.
 * - Errors: every call returns amg_status; nothing throws across the ABI.
 *   Arguments are validated on the host before any launch.  A thread-local
 *   message with details is available from amg_last_error().
 * - Handles are not thread-safe; distinct handles may be used from distinct
 *   threads.
 */
#ifndef AMG_H
#define AMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMG_OK = 0,
  AMG_ERR_ARG = 1,     /* invalid argument (NULL, out of range, non-finite) */
  AMG_ERR_SHAPE = 2,   /* lattice / block / layout mismatch                 */
  AMG_ERR_NAN = 3,     /* non-finite values detected                         */
  AMG_ERR_NOMEM = 4,   /* device allocation failed                           */
  AMG_ERR_HIP = 5,     /* a HIP runtime call failed                          */
  AMG_ERR_RANK = 6,    /* block near-null vectors are linearly dependent     */
  AMG_ERR_NOCONV = 7,  /* solver hit max_iter; psi holds the best iterate    */
  AMG_ERR_STATE = 8,   /* call not valid for this handle's state             */
  AMG_ERR_SINGULAR = 9 /* the coarsest operator of an exact solve is singular */
} amg_status;

typedef enum { AMG_F64 = 0, AMG_F32 = 1 } amg_prec;  /* complex<double>, complex<float> */

typedef struct amg_gauge amg_gauge;
typedef struct amg_solver amg_solver;

typedef struct {
  int nd;        /* 2 (U(1), Schwinger model) or 4 (SU(3)) */
  int dims[4];   /* L_1..L_nd; even extents; dims[nd..3] ignored */
} amg_lattice;

/* Multigrid parameters.  Defaults (amg_default_params) are the paper's where
 * it gives one: 4x4 blocks, M = 8 vectors, omega = 0.8, 2 + 2 smoothing
 * (numerical-test section). */
typedef struct {
  int nlevels;          /* 2..4 */
  int block[3][4];      /* block extents of coarsening l (fine level l -> l+1) */
  int nvec[3];          /* N_v of coarsening l; coarse dof per site = 2*N_v    */
  int nu_pre, nu_post;  /* MR smoothing steps before / after the coarse correction */
  double omega;         /* MR under-relaxation                                   */
  double coarse_tol;    /* coarsest GCR: stop when |r| <= coarse_tol |b|         */
  int coarse_maxiter;   /* coarsest GCR iteration cap                            */
  int coarse_restart;   /* coarsest GCR restart length (<= 32)                   */
  int outer_restart;    /* fine FGCR restart length (<= 32)                      */
  int inner_prec;       /* AMG_F64: FP64 V-cycle; AMG_F32: FP32 V-cycle          */
  int p_bf16;           /* with AMG_F32: store P in bfloat16 (Galerkin uses the rounded P) */
  double kcycle_tol;    /* intermediate levels: flexible GCR preconditioned by their own cycle */
  int kcycle_maxiter;   /*   to kcycle_tol, at most kcycle_maxiter (<= 32) steps; 0: V-cycle */
  int coarse_dense_max; /* a coarsest level of at most this many unknowns (V * 2 nvec of the finished
                         * level, <= AMG_DENSE_MAX; the adaptive setup's partially built levels follow
                         * the finished level) is solved exactly: the recursion of the V-cycle ends in a direct solve
                         * (the five-step list before Eq. (3)).  The dense matrix of its Galerkin
                         * operator is inverted at setup (and after a mass change) by Gauss-Jordan
                         * elimination with partial pivoting in FP64 (AMG_ERR_SINGULAR if a pivot
                         * is zero); each coarsest solve is then one dense matrix-vector product
                         * (FP32 copy of the inverse for the FP32 cycle).  Larger coarsest levels
                         * use GCR (coarse_tol, coarse_maxiter, coarse_restart).  Default 4096.
                         * Batched solves (amg_batch_create) use GCR on every instance. */
  int coarse_jacobi;    /* 1: the coarsest GCR (where not dense) is right-preconditioned by the
                         * inverse M of each coarse site's diagonal block (levels of at most 48 dof
                         * per site): GCR runs on the stencil of D_hat M, built at setup and after
                         * a mass change, and the result is M y.  Its iterates are those of GCR
                         * with the fixed preconditioner z = M r.  A level whose diagonal block is
                         * singular keeps the plain GCR.  Not applied inside batched solves.
                         * Default 0. */
  int coarse_eo;        /* 1 (with coarse_jacobi, on 2d levels with even extents): that GCR runs on
                         * the even sites only: with T = D_hat M split by site parity (unit
                         * diagonal), (1 - T_eo T_oe) y_e = b_e - T_eo b_o to |r_e| <= coarse_tol |b|
                         * (the odd residual is zero), then y_o = b_o - T_oe y_e and x = M y.
                         * Default 0. */
} amg_mg_params;

#define AMG_DENSE_MAX 8192

typedef struct {
  int iters;                 /* outer FGCR (or CG) iterations                  */
  int converged;             /* true residual <= tol                           */
  double true_rel_res;       /* |chi - D psi| / |chi|, FP64, recomputed       */
  long long n_fine_D;        /* fine D applications (all precisions)          */
  long long n_fine_Ddag;     /* fine D^dagger applications                    */
  long long n_coarse;        /* coarse-level operator applications            */
  double t_ms;               /* wall time of the call (host clock, synchronised) */
} amg_solve_info;

/* ---- errors ------------------------------------------------------------ */
const char* amg_status_str(amg_status s);
const char* amg_last_error(void);   /* thread-local detail of the last failure */

/* ---- device memory -------------------------------------------------------
 * Library plumbing (no passage of the paper defines it).  From this call on,
 * the internal device buffers of every handle (gauge copies, hierarchies,
 * work vectors, batches, networks) are taken from alloc(bytes, stream, ctx),
 * which returns a device pointer or NULL (the call that needed the memory
 * then fails with AMG_ERR_NOMEM), and handed back to release(ptr, stream,
 * ctx); stream is NULL (the buffers are used on whatever stream a call
 * names).  A buffer goes back to the routines that allocated it, also after
 * a later amg_set_allocator; before handing one back the library waits for
 * the device to finish its queued work, so a caching allocator may give the
 * block out again at once.  alloc = release = NULL restores hipMalloc /
 * hipFree; exactly one of them NULL is AMG_ERR_ARG.  Process-wide; do not
 * call it while another thread creates or grows handles. */
amg_status amg_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                             void (*release)(void* ptr, void* stream, void* ctx), void* ctx);

/* ---- gauge field and the fine operator --------------------------------- */

/* Copy links (canonical complex128, [nd][V][nc][nc]) into a new gauge handle
 * with FP64 and FP32 internal copies (structure-of-arrays).  mass is m of
 * the operator (d + m) - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) delta_{x+mu,y}
 * + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y}] (definition after Eq. (1);
 * diagonal read as d + m).  Synchronises `stream` before returning. */
amg_status amg_gauge_create(const amg_lattice* lat, const void* dev_links, double mass,
                            void* stream, amg_gauge** out);
amg_status amg_gauge_set_mass(amg_gauge* g, double mass);
/* Dimension, extents and link storage of a handle (library plumbing, no
 * passage of the paper defines it).  links_compressed = 1: every 4d link was
 * in SU(3) (unitary, unit determinant, to 1e-9) at creation, and the stencil
 * reads the first two rows of each link and rebuilds the third as the
 * conjugated cross product of the first two; 0: full 3 x 3 links.  Any
 * pointer may be NULL. */
amg_status amg_gauge_info(const amg_gauge* g, int* nd, int* dims4, int* links_compressed);
amg_status amg_gauge_destroy(amg_gauge* g);

/* dev_out = D dev_in (dagger = 0) or D^dagger dev_in (dagger = 1), nrhs
 * canonical fields of precision prec (complex128 or complex64).  In-place
 * (dev_out == dev_in) is an error.  Computes in prec. */
amg_status amg_apply(const amg_gauge* g, int dagger, int prec, const void* dev_in,
                     void* dev_out, int nrhs, void* stream);

/* As amg_apply, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the call allocates nothing.  The two layout conversions are staged in a
 * fixed device array of 64 MiB (each GPU the library runs on holds its own
 * copy until the process ends) instead of the handle's buffers, so
 * 2 * V * dof * nrhs complex numbers of precision prec (each half rounded up
 * to 256 bytes) must fit in 64 MiB, else AMG_ERR_ARG before any launch.  Same
 * kernels and results as amg_apply.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race.
 * The current device must be the one the gauge handle was created on
 * (AMG_ERR_STATE). */
amg_status amg_apply_noalloc(const amg_gauge* g, int dagger, int prec, const void* dev_in,
                             void* dev_out, int nrhs, void* stream);

/* Apply the fine stencil `iters` times on the handle's internal
 * structure-of-arrays buffers (no layout conversion): the kernel that the
 * solver runs, for bandwidth measurement.  Enqueued on `stream`. */
amg_status amg_apply_internal(amg_gauge* g, int dagger, int prec, int nrhs, int iters,
                              void* stream);

/* CG on the normal equations (the paper's baseline): D^dag D psi = D^dag chi
 * in FP64, stopping on |chi - D psi| <= tol |chi|.  info: one per call. */
amg_status amg_cgnr_solve(const amg_gauge* g, const void* dev_chi, void* dev_psi,
                          double tol, int max_iter, amg_solve_info* info, void* stream);

/* ---- multigrid ---------------------------------------------------------- */
void amg_default_params(amg_mg_params* p);

/* Build the hierarchy from given near-null vectors (Eq. (5) and the text
 * after it): dev_nullvecs[l] holds nvec[l] complex128 fields of level l in
 * canonical layout, [nvec][V_l][dof_l].  Blocks are orthonormalised per
 * chirality in FP64 (AMG_ERR_RANK on dependence), coarse operators are the
 * Galerkin products P^dag D P (Eq. (2)).  Synchronises `stream`. */
amg_status amg_setup(const amg_gauge* g, const amg_mg_params* p,
                     const void* const* dev_nullvecs, void* stream, amg_solver** out);

/* Adaptive setup (text from Eq. (4) to the recursion remark after Eq. (5)),
 * level by level: vector 1 is dev_init[l][0] relaxed by nu0 MR steps on
 * A_l v = 0; vector k > 1 is dev_init[l][k-1] after ncyc sweeps of the
 * two-level error propagation e <- e - V(A_l e) with the k-1 vectors built
 * so far.  dev_init[l]: nvec[l] random complex128 fields of level l
 * (canonical).  Synchronises `stream`. */
amg_status amg_setup_adaptive(const amg_gauge* g, const amg_mg_params* p,
                              const void* const* dev_init, int nu0, int ncyc,
                              void* stream, amg_solver** out);

/* As amg_setup_adaptive with per-coarsening counts nu0[l], ncyc[l]. */
amg_status amg_setup_adaptive_levels(const amg_gauge* g, const amg_mg_params* p,
                                     const void* const* dev_init, const int* nu0, const int* ncyc,
                                     void* stream, amg_solver** out);

/* Reuse the setup at another fine mass: every level's diagonal shifts by
 * (mass - current) P^dag ... P 1 P ... P (exact, also for a rounded P). */
amg_status amg_solver_set_mass(amg_solver* s, double mass);
amg_status amg_solver_destroy(amg_solver* s);

/* Solve D psi = chi for nrhs canonical complex128 fields by FP64 flexible GCR
 * preconditioned by one V-cycle per iteration, to |chi - D psi| <= tol |chi|
 * (true FP64 residual).  info: array of nrhs.  Returns AMG_ERR_NOCONV if any
 * right-hand side misses tol within max_iter (psi holds the last iterate),
 * AMG_ERR_NAN (before any iteration, psi unwritten) if a right-hand side has
 * a non-finite entry.  Synchronises `stream` once per outer iteration. */
amg_status amg_solve(amg_solver* s, const void* dev_chi, void* dev_psi, int nrhs,
                     double tol, int max_iter, amg_solve_info* info, void* stream);

/* ---- building blocks, exposed for parity checks -------------------------- */

/* Raw near-null vectors of coarsening `level` as stored (before block
 * orthonormalisation), complex128 canonical [nvec][V_l][dof_l]. */
amg_status amg_get_nullvecs(const amg_solver* s, int level, void* dev_out, void* stream);

/* Coarse operator of level `level` >= 1 in FP64: dev_out[V_l][2nd+1][Nc][Nc]
 * complex128, block 0 the diagonal, block 1+2mu the coupling to x+mu,
 * block 2+2mu to x-mu, row-major [t][t'] (row = output dof). */
amg_status amg_get_coarse_op(const amg_solver* s, int level, void* dev_out, void* stream);

/* Apply the operator of `level` (0 = fine) in precision prec to nrhs
 * canonical fields of that level's precision. */
amg_status amg_level_apply(const amg_solver* s, int level, int dagger, int prec,
                           const void* dev_in, void* dev_out, int nrhs, void* stream);

/* Restriction r_hat = P^dag r (dir = 0) or prolongation e = P e_hat (dir = 1)
 * between level `level` and level+1 (the transfers of the five-step V-cycle
 * before Eq. (3), P built as in Eq. (5)), nrhs canonical fields.
 * prec = AMG_F64: FP64 P and complex128 fields; AMG_F32: the P that the FP32
 * cycle uses (FP32, or bfloat16 with p_bf16) and complex64 fields,
 * accumulation in FP32 (AMG_ERR_STATE for a solver with inner_prec = AMG_F64). */
amg_status amg_transfer(const amg_solver* s, int level, int dir, int prec, const void* dev_in,
                        void* dev_out, int nrhs, void* stream);

/* The prolongator of coarsening `level` as stored (Eq. (5) with the chirally
 * split, block-orthonormalised vectors): dev_out[V_l][dof_l][2 nvec_l]
 * complex128, row (site, component), column t = chi*N_v + k, zero where the
 * component's chirality is not chi.  prec = AMG_F64: the FP64 P; AMG_F32:
 * the FP32 cycle's copy (FP32 or bfloat16 values, widened exactly). */
amg_status amg_get_prolongator(const amg_solver* s, int level, int prec, void* dev_out, void* stream);

/* One V-cycle x = V(b) from the finest level, in the solver's inner
 * precision; b and x canonical complex128, nrhs fields. */
amg_status amg_vcycle(amg_solver* s, const void* dev_b, void* dev_x, int nrhs, void* stream);

/* nu MR steps (omega from the params) on level `level` from x = 0:
 * x = MR_nu(b) in precision prec, b and x canonical fields of that
 * precision (complex128 / complex64), nrhs of them.  AMG_F32 needs a solver
 * built with inner_prec = AMG_F32 (else AMG_ERR_STATE). */
amg_status amg_mr(amg_solver* s, int level, int prec, int nu, const void* dev_b, void* dev_x,
                  int nrhs, void* stream);

/* ---- batched solves ---------------------------------------------------------
 * Many independent solves (different gauge fields, lattice sizes, masses)
 * advanced together: every stage of the outer iteration is one launch over
 * all instances (instance = grid z), and the stages of each outer-iteration
 * step are captured once into a HIP graph and replayed.  Right-hand sides
 * that have converged are masked on the device. */
typedef struct amg_batch amg_batch;

/* Group n solvers (two-dimensional, same hierarchy depth, dof per level and
 * solver parameters); instance i solves nrhs[i] right-hand sides.  With
 * autotune != 0 the launch shapes are chosen jointly by timing one batched
 * outer step per candidate: the grid of the reducing kernels (128, 256, 512,
 * 1024 blocks) x the coarse stencil (the multi-rhs MFMA kernel for every
 * instance, or one right-hand side per grid row); amg_batch_tuning reports
 * every candidate.  Without autotune: 1024 blocks and the MFMA kernel (or the
 * per-rhs stencil when the environment sets AMG_BATCH_MRHS=0).  The solvers
 * must outlive the batch and must not be used concurrently with it. */
amg_status amg_batch_create(amg_solver* const* solvers, const int* nrhs, int n, int autotune, void* stream,
                            amg_batch** out);
/* Solve all instances to |chi - D psi| <= tol |chi| (true FP64 residual per
 * right-hand side).  dev_chi[i], dev_psi[i]: nrhs[i] canonical complex128
 * fields of instance i.  info: sum(nrhs) entries, instance-major.  Returns
 * AMG_ERR_NOCONV if any right-hand side misses tol, AMG_ERR_NAN (before any
 * iteration) if one has a non-finite entry.  Synchronous. */
amg_status amg_batch_solve(amg_batch* b, const void* const* dev_chi, void* const* dev_psi, double tol,
                           int max_iter, amg_solve_info* info, void* stream);
/* The autotuned reduction grid cap and the number of batched launches per outer step. */
amg_status amg_batch_info(const amg_batch* b, int* red_cap, int* stages_per_iteration);
/* The same, with the coarse-stencil choice (1: multi-rhs MFMA kernel, 0: per-rhs stencil). */
amg_status amg_batch_info2(const amg_batch* b, int* red_cap, int* mrhs, int* stages_per_iteration);
/* The autotuner's candidates in the order timed: reduction grid cap, coarse
 * stencil choice and ms per batched outer iteration, at most max entries
 * written; returns the number of candidates (0 without autotune, -1 for a
 * NULL batch). */
int amg_batch_tuning(const amg_batch* b, int max, int* red_cap, int* mrhs, float* ms_per_iteration);
amg_status amg_batch_destroy(amg_batch* b);

/* ---- kernel timing (HIP events) -------------------------------------------
 * While enabled, every launch of kernel `kind` on level `level` made by this
 * solver is timed by a pair of HIP events that the launch itself stamps at
 * the start and end of the kernel's execution (hipExtLaunchKernelGGL), on
 * its stream.  amg_profile_read
 * synchronises on the last event and returns the summed kernel time and the
 * number of launches since enabling.  kind: 0 fine Wilson stencil, 1 coarse
 * block stencil, 2 restriction, 3 prolongation (level = the fine side),
 * 4 coarse block stencil with the MR epilogue only, 5 even-odd half-lattice
 * hop, 6 even-odd reduced operator (9-point stencil of the even sites). */
amg_status amg_profile_enable(amg_solver* s, int kind, int level, int enable);
amg_status amg_profile_read(amg_solver* s, double* total_ms, long long* launches);
/* kind = -1 and / or level = -1 in amg_profile_enable time every kind / level
 * (kind 1 then excludes the launches counted as kind 4); this returns the
 * part of the recorded launches of one (kind, level). */
amg_status amg_profile_read_kind(amg_solver* s, int kind, int level, double* total_ms, long long* launches);

/* Introspection: lattice extents and dof per site of a level. */
amg_status amg_level_info(const amg_solver* s, int level, int* dims4, int* dof, long long* V);

/* Convergence factor of the multigrid method as a stationary iteration,
 * e <- e - M(D e) with M one V-cycle (the test of the adaptive construction,
 * text after Eq. (5): a random error either decays quickly or survives).
 * Starts from the canonical complex128 fine field dev_e0 (not modified),
 * runs `iters` >= 1 iterations and returns
 * rho = (|e_iters| / |e_0|)^(1/iters).  Synchronous. */
amg_status amg_mg_convergence(amg_solver* s, const void* dev_e0, int iters, double* rho, void* stream);

/* ---- learned setup (two-dimensional U(1) only) -------------------------------
 * A local convolutional network proposes the initial near-null vectors of
 * the finest coarsening, which the adaptive procedure (Eq. (4) and the text
 * after Eq. (5)) then refines.  The network is not part of the paper; it is
 * trained on near-null vectors that the adaptive setup itself produced.
 *
 * Network: four 3x3 convolutions with periodic padding, channels
 * 4 -> 64 -> 64 -> 64 -> 32, tanh after the first three.  Input per site:
 * (cos, sin) of both link angles after a block-local tree gauge fixing
 * (4x4 blocks; the x_1 links along every block row and the x_2 links along
 * the first block column are set to 1 by g = exp(i phi), phi = 0 at the
 * block origin).  Output channel 4k + 2s + c is component c (re, im) of spin
 * s of proposal k = 0..7 in the fixed gauge; proposals are returned in the
 * original gauge, v = g^dag v'.
 *
 * Parameters (amg_cnn_num_params() floats, 94,688): for each layer the
 * weights W[c_out][c_in][3][3] (y(i,j) += W[o][c][di][dj] x(i+di-1, j+dj-1),
 * i = x_2 row, j = x_1 column) then the biases b[c_out].  FP32 master copy
 * with Adam moments; activations and the compute copy of the weights in
 * bfloat16 (bf16 != 0) or FP32, accumulation in FP32.
 *
 * Loss (mean over configurations, 4x4 blocks, spin s and targets k): with V
 * the 16 x 8 block restriction of the predictions of spin s and t_k the
 * normalised block restriction of target k, 1 - t_k^dag V (V^dag V + 1e-3)^-1 V^dag t_k,
 * i.e. how much of each target lies outside the predicted block span (the
 * prolongator of Eq. (5) only depends on that span).  Evaluated in FP64.
 *
 * Links: dev_links[b] is one configuration in the canonical gauge layout,
 * [B][2][L2*L1] complex128 of unit modulus.  Targets: dev_vecs[b][8][L2*L1][2]
 * complex128 canonical (what amg_get_nullvecs returns for level 0).  L1, L2
 * multiples of 16.  Calls with gradients or training synchronise `stream`. */
typedef struct amg_cnn amg_cnn;
long long amg_cnn_num_params(void);
amg_status amg_cnn_create(const float* host_params, int bf16, amg_cnn** out);
amg_status amg_cnn_destroy(amg_cnn* n);
amg_status amg_cnn_get_params(const amg_cnn* n, float* host_out);
amg_status amg_cnn_set_params(amg_cnn* n, const float* host_params);
/* Network output for B configurations, dev_out[B][32][L2][L1] float32. */
amg_status amg_cnn_forward(amg_cnn* n, const void* dev_links, int B, int L1, int L2, float* dev_out, void* stream);
/* Mean loss and (host_grads != NULL) its gradient, amg_cnn_num_params() floats
 * in parameter order; parameters unchanged. */
amg_status amg_cnn_loss_grad(amg_cnn* n, const void* dev_links, const void* dev_vecs, int B, int L1, int L2,
                             double* loss, float* host_grads, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean loss of the
 * batch; returns the loss before the step.  AMG_ERR_NAN leaves the
 * parameters unchanged. */
amg_status amg_cnn_train_step(amg_cnn* n, const void* dev_links, const void* dev_vecs, int B, int L1, int L2,
                              float lr, double* loss, void* stream);
/* 8 proposals for one configuration, dev_vecs_out[8][L2*L1][2] complex128. */
amg_status amg_cnn_propose(amg_cnn* n, const void* dev_links, int L1, int L2, void* dev_vecs_out, void* stream);

/* Setup from given starting vectors for the finest coarsening (e.g. the
 * network's proposals).  Level 0: vectors 0..n_start-1 are the first n_start
 * canonical complex128 fields of dev_start0 ([n][V][dof]), each relaxed by
 * nu_ref MR steps on D v = 0 (Eq. (4)); vectors n_start..nvec[0]-1 come from
 * one adaptive iteration each (text after Eq. (5)): dev_init[0][k - n_start]
 * after ncyc_ref sweeps of the two-level error propagation e <- e - V(D e)
 * built from the vectors before it.  Deeper coarsenings l >= 1: adaptive
 * setup from dev_init[l] with (nu0, ncyc).  1 <= n_start <= nvec[0].
 * Synchronous. */
amg_status amg_setup_refined(const amg_gauge* g, const amg_mg_params* p, const void* dev_start0,
                             int n_start, int nu_ref, int ncyc_ref, const void* const* dev_init,
                             int nu0, int ncyc, void* stream, amg_solver** out);

/* Learned setup: amg_setup_refined from the network's proposals for g's
 * links (n_start <= 8 of them).  If that fails (dependent vectors, non-finite
 * values) or, with rho_iters > 0, the convergence factor of the resulting
 * method measured from dev_init[0][0] over rho_iters iterations
 * (amg_mg_convergence) exceeds rho_max, the plain adaptive setup from
 * dev_init with (nu0, ncyc) is built instead and *fell_back is set to 1.
 * *rho gets the factor of the returned hierarchy (-1 when not measured).
 * Synchronous. */
amg_status amg_setup_learned(const amg_gauge* g, const amg_mg_params* p, amg_cnn* net,
                             const void* const* dev_init, int n_start, int nu_ref, int ncyc_ref,
                             double rho_max, int rho_iters, int nu0, int ncyc, void* stream,
                             amg_solver** out, int* fell_back, double* rho);

/* ---- multigrid for the normal equations A = D^dag D (2d) ----------------
 * The paper's own variant (numerical-test section): the Galerkin hierarchy
 * A_{l+1} = P_l^dag A_l P_l (Eq. (2)) of the Hermitian positive definite
 * A_0 = D^dag D, with one coarse degree of freedom per near-null vector (no
 * chiral split), P_l the block-orthonormalised vectors (Eq. (5)) optionally
 * smoothed by one damped Richardson step ("smoothed aggregation", adaptive-
 * method section), the degree-2 smoother whose two minimal-residual step
 * lengths are computed once and then frozen (R = R^dag), the V-cycle of the
 * five steps before Eq. (3) ending in an exact solve, and conjugate gradients
 * preconditioned by one V-cycle per iteration (MG-CG).
 * Every coarse operator is a 9-point box stencil of M x M blocks (D^dag D
 * couples a site to its 3 x 3 box only: for r = 1 the straight double hop
 * cancels), built by probing with coloured unit vectors: coarse extents must
 * be >= 3 and have a divisor >= 3 (period of the colouring); with smoothing,
 * blocks >= 3 (the widened columns then still couple neighbouring blocks
 * only) and coarse extents with a divisor >= 2.
 * Field layouts: fine fields [site][2] complex128 (x_1 fastest); coarse
 * fields [site][M]; near-null vectors [M][V_l][dof_l].  All FP64.
 * Handles keep a pointer to their gauge (which must outlive them) and run on
 * its device; calls on one handle must not overlap.  Synchronous. */
typedef struct amg_normal amg_normal;

typedef struct {
  int nlevels;            /* 2..4 (levels including the finest)                        */
  int block[3][2];        /* block extents of coarsening l                              */
  int nvec[3];            /* M of coarsening l (1..16): coarse dof per site             */
  double omega;           /* under-relaxation of the frozen MR steps (paper: 0.8)       */
  double sa_factor;       /* f > 0: P = (1 - f / lambda_l A_l) P_tent, lambda_l the     */
                          /* Rayleigh quotient of A_l after power_steps power steps     */
                          /* from the level's smoother vector; 0: unsmoothed P          */
  int power_steps;        /* default 20                                                  */
  int coarse_dense_max;   /* the coarsest level (V M unknowns) must not exceed this: its */
                          /* dense Galerkin matrix is inverted (Gauss-Jordan, partial    */
                          /* pivoting); <= AMG_DENSE_MAX, default 4096                   */
  int fine_box;               /* 1: A_0 = D^dag D also stored as a 9-point stencil of 2 x 2 */
                              /* blocks (probed per mass) and applied in one launch, on    */
                              /* lattices up to 2^18 sites; 0: always D then D^dag         */
  int setup_dense_max;        /* adaptive set-up: a set-up cycle's coarse level of at most */
                              /* this many unknowns is solved exactly (dense inverse),    */
  double setup_coarse_tol;    /* a larger one by CG to setup_coarse_tol (at most          */
  int setup_coarse_maxiter;   /* setup_coarse_maxiter iterations); defaults 1024, 1e-6    */
} amg_normal_params;

typedef struct {
  int iters;                 /* CG iterations                                             */
  int converged;             /* |b - A psi| <= tol |b|, b = D^dag chi, recomputed          */
  int restarts;              /* CG restarts on a recomputed residual                       */
  double rel_res_normal;     /* |b - A psi| / |b|, FP64                                   */
  double rel_res_D;          /* |chi - D psi| / |chi|, FP64                               */
  long long n_fine_D;        /* fine D applications in the call                            */
  long long n_fine_Ddag;     /* fine D^dag applications in the call                        */
  double t_ms;               /* wall time of the call (synchronised)                       */
} amg_normal_info;

void amg_normal_default_params(amg_normal_params* p);

/* Hierarchy from given near-null vectors: dev_vecs[l] holds the nvec[l]
 * vectors of coarsening l ([M][V_l][dof_l] complex128), dev_sb[l] one field
 * of level l ([V_l][dof_l]) from which the frozen step lengths (and the power
 * estimate of the smoothing damping) are computed.  The mass is g's current
 * mass.  AMG_ERR_RANK if a block's vectors are linearly dependent,
 * AMG_ERR_SINGULAR if the coarsest matrix is, AMG_ERR_SHAPE for extents the
 * probing cannot colour. */
amg_status amg_normal_setup(const amg_gauge* g, const amg_normal_params* p, const void* const* dev_vecs,
                            const void* const* dev_sb, void* stream, amg_normal** out);

/* Adaptive hierarchy (text from Eq. (4) to the recursion remark after Eq. (5)),
 * coarsening by coarsening: vector 0 is dev_init[l][0] after nu0[l] MR steps
 * (omega) on A_l v = 0; vector k >= 1 is dev_init[l][k] after ncyc[l] sweeps
 * of e <- e - V(A_l e), V the two-level cycle built from vectors 0..k-1
 * (coarse level solved exactly up to setup_dense_max unknowns, else by CG),
 * normalised. */
amg_status amg_normal_setup_adaptive(const amg_gauge* g, const amg_normal_params* p, const void* const* dev_init,
                                     const void* const* dev_sb, const int* nu0, const int* ncyc, void* stream,
                                     amg_normal** out);

/* Rebuild P (smoothing), every Galerkin product, the step lengths and the
 * coarsest inverse for D(mass) from the same near-null vectors (the set-up
 * at the lightest mass reused for heavier ones, numerical-test section). */
amg_status amg_normal_set_mass(amg_normal* S, double mass, void* stream);

/* Solve D^dag D psi = D^dag chi by CG (precond 0) or MG-CG (precond 1) from
 * psi = 0, until the recursive residual of the normal equations falls below
 * tol |D^dag chi| and the recomputed one confirms it (else restart from the
 * recomputed residual).  AMG_ERR_NOCONV after max_iter iterations (psi holds
 * the last iterate). */
amg_status amg_normal_solve(amg_normal* S, const void* dev_chi, void* dev_psi, double tol, int max_iter,
                            int precond, amg_normal_info* info, void* stream);

/* dev_out = V dev_in: one V-cycle of the finest level (fine fields). */
amg_status amg_normal_vcycle(amg_normal* S, const void* dev_in, void* dev_out, void* stream);

/* dev_out = A_level dev_in (level 0: D^dag D; level >= 1: the box stencil). */
amg_status amg_normal_level_apply(amg_normal* S, int level, const void* dev_in, void* dev_out, void* stream);

/* Exports (test infrastructure):
 *   what 0: P of coarsening `level` as the dense matrix [V_l dof_l][V_{l+1} M]
 *   what 1: A_level (level >= 1) as the dense matrix [V M][V M]
 *   what 2: the near-null vectors of coarsening `level` ([M][V_l][dof_l])
 * (row-major complex128, at most 2^28 entries, else AMG_ERR_ARG). */
amg_status amg_normal_export(amg_normal* S, int level, int what, void* dev_out, void* stream);

/* Level facts: extents, dof per site, the frozen step lengths (tau0, tau1) of
 * the level's smoother, and (lambda, omega_sa) of its smoothed P (zeros on
 * the coarsest level or without smoothing).  NULL outputs are skipped. */
amg_status amg_normal_level_info(const amg_normal* S, int level, int* dims2, int* dof, double* taus2,
                                 double* lambda_omega2);

amg_status amg_normal_destroy(amg_normal* S);

#ifdef __cplusplus
}
#endif
#endif /* AMG_H */
