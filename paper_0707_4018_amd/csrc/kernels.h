// Launchers of the gfx950 kernels (host-callable), shared by the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace amg {

// epilogues fused into operator applications
enum Epi {
  EPI_PLAIN = 0,  // out = A in
  EPI_MRDOT = 1,  // out = A in; alpha = omega <out, in> / <out, out>  -> scal[slot + 2 rhs]
  EPI_RESID = 2,  // out = b - A in
  EPI_NORM = 3,   // out = A in; scal[slot + rhs] = <out, out>
  EPI_MRPART = 4  // out = A in; this block's <out, in> (re, im), <out, out> -> part[(3 rhs + q) nblk + block]
};

constexpr int RED_MAX_BLOCKS = 1024;   // largest grid of kernels that reduce
static_assert(RED_MAX_BLOCKS <= RED_BLOCKS_LIMIT, "ticket layout covers at most RED_BLOCKS_LIMIT blocks");
// grid cap used when launching reducing kernels (<= RED_MAX_BLOCKS); a launch
// shape chosen by the batch autotuner, 1024 by default
int red_block_cap();
void set_red_block_cap(int cap);
constexpr int GCR_KMAX = 32;           // longest GCR restart cycle

// Reduction plumbing handed to every kernel that reduces or can skip rhs.
struct RedArgs {
  double* part = nullptr;      // partial sums scratch
  unsigned* ticket = nullptr;  // per-rhs arrival counters, TICKETS_PER_RHS each (zero between launches)
  double* scal = nullptr;      // solver scalars
  int slot = 0;                // where this reduction writes in scal
  double omega = 1.0;          // MR under-relaxation (EPI_MRDOT)
  const int* flags = nullptr;  // per-rhs skip flags (nullptr: none)
};

__device__ __forceinline__ void finalize_mr(const double* tot, const RedArgs& r, int rhs) {
  const double pp = tot[2];
  const double s = pp > 0.0 ? r.omega / pp : 0.0;
  gptr<double> scal = gl(r.scal);
  scal[r.slot + 2 * rhs] = s * tot[0];
  scal[r.slot + 2 * rhs + 1] = s * tot[1];
}

template <typename T>
struct WilsonArgs {
  cplx<T>* out = nullptr;
  const cplx<T>* in = nullptr;
  const cplx<T>* b = nullptr;       // EPI_RESID
  cplx<T>* copy_out = nullptr;      // optional copy of `in`
  const cplx<T>* U = nullptr;       // internal link layout of precision T
  // 4d only: the SU(3) links as their first two rows (third row rebuilt as
  // the conjugated cross product), or nullptr: FP32 [mu][3][site] float4
  // (u00 u01 | u02 u10 | u11 u12), FP64 [mu][6][site] double2
  const void* Uc = nullptr;
  double mass = 0.0;
  int L1 = 0, L2 = 0, L3 = 1, L4 = 1;
  int nrhs = 1;
  RedArgs red;
};

template <typename T> void launch_wilson2d(const WilsonArgs<T>& a, int dagger, int epi, hipStream_t st);
template <typename T> void launch_wilson4d(const WilsonArgs<T>& a, int dagger, int epi, hipStream_t st);
void launch_wilson2d_split(double2* out, const double2* in, const double2* U, double mass, int L1,
                           int L2, int b1, int b2, int nrhs, hipStream_t st);
void launch_wilson4d_split(double2* out, const double2* in, const double2* U, double mass,
                           const int* dims, const int* blk, int nrhs, hipStream_t st);

// ---- coarse block stencil ---------------------------------------------------
struct CoarseGeom {
  int nd;
  int dims[4];
  long V;
  int nc;       // dof per site
};

template <typename T>
struct CoarseArgs {
  cplx<T>* out = nullptr;
  const cplx<T>* in = nullptr;
  const cplx<T>* b = nullptr;
  cplx<T>* copy_out = nullptr;
  const cplx<T>* Y = nullptr;   // [V][2nd+1][nc (col)][nc (row)]
  CoarseGeom g;
  int nrhs = 1;
  RedArgs red;
};
template <typename T> void launch_coarse(const CoarseArgs<T>& a, int dagger, int epi, hipStream_t st);
// blocks of the N_c = 16 stencil launched with a reducing epilogue (partial sums per block)
int coarse16_red_blocks(long V);
// many right-hand sides per launch on MFMA (FP32; N_c = 16 or 48; plain or residual epilogue)
bool coarse_mrhs_supported(int nc, int epi);
void launch_coarse_mrhs(const CoarseArgs<float>& a, int dagger, int epi, hipStream_t st);
// fused GCR step for N_c = 16 levels: part 1 (apply + all sums) and part 2 (updates)
template <typename T>
void launch_gcr16_apply_dots(const CoarseArgs<T>& a, const cplx<T>* r, const cplx<T>* Wb, long dstride, int k,
                             int beta_slot, int ww_slot, int alpha_slot, hipStream_t st);
// (rr_slot < 0: no <r, r> reduction and no flag)
template <typename T>
void launch_gcr_update2(cplx<T>* x, cplx<T>* r, const cplx<T>* zsrc, cplx<T>* Wb, cplx<T>* Zb, long dstride, int k,
                        long n, int nrhs, RedArgs red, int beta_slot, int alpha_slot, int rr_slot, int bb_slot,
                        double tol2, int* set_flags, hipStream_t st);
void launch_coarse_split(double2* out, const double2* in, const double2* Y, const CoarseGeom& g,
                         const int* blk, int nrhs, hipStream_t st);
void launch_coarse_massmat(double2* out, const double2* in, const double2* M, const CoarseGeom& g,
                           int nrhs, hipStream_t st);

// ---- exact coarsest solve (dense inverse) ----------------------------------------
// A[N][N] (N = V nc, row-major) = the dense matrix of the block stencil Y
void launch_dense_assemble(double2* A, const double2* Y, const CoarseGeom& g, hipStream_t st);
// Gauss-Jordan inversion with partial pivoting of A (overwritten; B: second
// N x N buffer).  key: N+1 u64, piv / used / pinv: N ints, err: 2 ints
// (err[0] != 0 afterwards: singular).  Ainv32 may be NULL.
void launch_gj_invert(double2* A, double2* B, long N, unsigned long long* key, int* piv, int* used, int* pinv,
                      int* err, double2* Ainv, float2* Ainv32, hipStream_t st);
// x[rhs] = Ainv b[rhs] (fields of N complex numbers per rhs)
template <typename T>
void launch_dense_apply(cplx<T>* x, const cplx<T>* b, const cplx<T>* Ainv, long N, int nrhs, const int* flags,
                        hipStream_t st);

// ---- transfers ----------------------------------------------------------------
struct TransferGeom {
  int nd;
  int fdims[4];   // fine extents
  int blk[4];     // block extents
  int cdims[4];   // coarse extents
  long Vf, Vc;
  int bs;         // sites per block
  int dof;        // fine dof per site
  int nv;         // vectors per chirality
  Layout lf;      // fine field layout
};
// P storage kinds
enum PKind { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };
template <typename T>
void launch_restrict(cplx<T>* out, const cplx<T>* in, const void* P, int pkind, const TransferGeom& g,
                     int nrhs, const int* flags, hipStream_t st);
template <typename T>
void launch_prolong(cplx<T>* out, const cplx<T>* in, const void* P, int pkind, const TransferGeom& g,
                    int nrhs, int accumulate, const int* flags, hipStream_t st);
// the stored P (any kind) as dense rows per fine site: out[Vf][dof][2 nv] complex128
void launch_p_export(double2* out, const void* P, int pkind, const TransferGeom& g, hipStream_t st);
// block orthonormalisation (FP64): vecs [nv][per_rhs] in layout g.lf -> P [Vc][bs][dof][nv]
void launch_orthonormalise(double2* P, const double2* vecs, const TransferGeom& g, int* err_flag,
                           hipStream_t st);
void launch_galerkin_scatter(double2* Y, const double2* R, long Vc, int nc, int nk, int t0, int chunk,
                             hipStream_t st);
void launch_unit_coarse(double2* E, long Vc, int nc, int t0, int chunk, hipStream_t st);
// per nc x nc block: out[row*nc + col] = in[col*nc + row]
void launch_block_transpose(double2* out, const double2* in, long nblocks, int nc, hipStream_t st);

// ---- BLAS-1 and conversions ----------------------------------------------------
template <typename Tin, typename Tout>
void launch_convert(cplx<Tout>* out, const cplx<Tin>* in, long V, int dof, int Win, int Wout, int nrhs,
                    hipStream_t st);
void launch_p_convert(void* out, int pkind, const double2* in, long n, hipStream_t st);
void launch_p_roundtrip_bf16(double2* P, long n, hipStream_t st);
template <typename T>
void launch_mr_update(cplx<T>* x, cplx<T>* r_out, const cplx<T>* r_in, const cplx<T>* p,
                      const double* alpha, long n, int nrhs, int first, int update_r, const int* flags,
                      hipStream_t st, const double* part = nullptr, int nblk = 0, double omega = 1.0);
template <typename T>
void launch_norm2(const cplx<T>* v, long n, int nrhs, RedArgs red, hipStream_t st);
// GCR building blocks; directions stored contiguously: W_j = Wb + j * dstride
// one-reduction GCR orthogonalisation: betas, <w',w'> and alpha (then launch_gcr_update2);
// rr_slot >= 0: also <r, r> of the current residual and the flag rr <= tol2 * bb
template <typename T>
void launch_gcr_dots(const cplx<T>* Wb, long dstride, const cplx<T>* w, const cplx<T>* r, int k, long n, int nrhs,
                     RedArgs red, int beta_slot, int ww_slot, int alpha_slot, int rr_slot, int bb_slot, double tol2,
                     int* set_flags, hipStream_t st);
template <typename T>
void launch_gcr_mdot(const cplx<T>* Wb, long dstride, const cplx<T>* w, int k, long n, int nrhs,
                     RedArgs red, int beta_slot, int ww_slot, hipStream_t st);
template <typename T>
void launch_gcr_maxpy(cplx<T>* w, cplx<T>* z, const cplx<T>* Wb, const cplx<T>* Zb, long dstride,
                      const cplx<T>* r, int k, long n, int nrhs, RedArgs red, int beta_slot, int ww_slot,
                      int alpha_slot, hipStream_t st);
template <typename T>
void launch_gcr_update(cplx<T>* x, cplx<T>* r, const cplx<T>* z, const cplx<T>* w, long n, int nrhs,
                       RedArgs red, int alpha_slot, int rr_slot, int bb_slot, double tol2, int* set_flags,
                       hipStream_t st);
// flags[rhs] = inherit[rhs] || scal[rr + rhs] <= tol2 * scal[bb + rhs]
void launch_set_flags(int* flags, const int* inherit, const double* scal, int rr_slot, int bb_slot, double tol2,
                      int nrhs, hipStream_t st);
// out[rhs] = scal[slot + rhs]
void launch_gather(double* out, const double* scal, int slot, int nrhs, hipStream_t st);
// dst = src (src == nullptr: zero), n complex per rhs
template <typename T>
void launch_fill(cplx<T>* dst, const cplx<T>* src, long n, int nrhs, hipStream_t st);
template <typename T>
void launch_axpy(cplx<T>* y, const cplx<T>* x, double are, double aim, long n, int nrhs, hipStream_t st);
template <typename T>
void launch_scale_inv_norm(cplx<T>* v, const double* nn, long n, int nrhs, hipStream_t st);
void launch_diag_shift(double2* Y, const double2* M, long V, int nc, int ndir, double dm, hipStream_t st);
// right block-Jacobi preconditioning of a coarse level (nc <= 48): Minv = the
// inverse of each site's diagonal block (err[0] set if one is singular), AM =
// the stencil of A M, and out = M in
bool block_jacobi_supported(int nc);
void launch_block_inverse(double2* Minv, const double2* Y, long V, int ndir, int nc, int* err, hipStream_t st);
void launch_jacobi_couplings(double2* AM, const double2* Y, const double2* Minv, const CoarseGeom& g, hipStream_t st);
template <typename T>
void launch_block_apply(cplx<T>* out, const cplx<T>* in, const cplx<T>* M, long V, int nc, int nrhs, hipStream_t st);
// even-odd reduction of the block-Jacobi system T = A M on 2d levels with
// even extents: coupling blocks split by parity, half-lattice hops
// (epi 0: sum, 1: b - sum, 2: b - b2 + sum) and x = M (y_e, y_o)
bool eo_supported(int nd, const int* dims, int nc);
void launch_eo_split(double2* Ce, double2* Co, const double2* T, int L1, int L2, int nc, hipStream_t st);
// (out2: optional second copy of the result; zero: optional half field set to zero)
template <typename T>
void launch_eo_hop(cplx<T>* out, const cplx<T>* in, const cplx<T>* b, const cplx<T>* b2, const cplx<T>* C, int L1,
                   int L2, int nc, int par, int in_full, int b_full, int epi, int nrhs, hipStream_t st,
                   cplx<T>* out2 = nullptr, cplx<T>* zero = nullptr);
// the reduced operator 1 - T_eo T_oe as a 9-point stencil of the even sites
// (blocks [h][9][col][row], FP64 from the FP64 couplings) and its apply for
// N_c = 16 (epi 0: sum, 1: b - sum)
void launch_eo_schur_build(double2* S9, const double2* Ce, const double2* Co, int L1, int L2, int nc, hipStream_t st);
template <typename T>
void launch_eo_s9(cplx<T>* out, const cplx<T>* in, const cplx<T>* b, const cplx<T>* S9, int L1, int L2, int epi,
                  int nrhs, hipStream_t st);
template <typename T>
void launch_eo_block_apply(cplx<T>* x, const cplx<T>* ye, const cplx<T>* yo, const cplx<T>* M, int L1, int L2, int nc,
                           int nrhs, hipStream_t st);
void launch_links4d_pack(double2* U64, float2* U32, const double2* canon, long V, hipStream_t st);
// two-row (12-real) copies of SU(3) links in FP64 and FP32; *not_su3 (zero on
// entry) becomes nonzero if some link is not unitary with unit determinant to 1e-9
void launch_links4d_compress(double2* Uc64, float4* Uc32, const double2* canon, long V, int* not_su3,
                             hipStream_t st);
// whole coarsest-level GCR (N_c = 16) in one cooperative launch
template <typename T>
hipError_t launch_gcr16_persistent(const cplx<T>* Y, const CoarseGeom& g, const cplx<T>* b, cplx<T>* x, cplx<T>* r,
                                   cplx<T>* Zb, cplx<T>* Wb, long dstride, int m, int maxiter, double tol2, int nrhs,
                                   int nblk, double* part, unsigned* bar, int* err, int* iters, hipStream_t st,
                                   bool cooperative);
int gcr16_partials_per_block();
// CG on the normal equations
void launch_cg_update(double2* x, double2* r, const double2* p, const double2* q, long n, int nrhs,
                      RedArgs red, int gamma_slot, int qq_slot, int rr_slot, hipStream_t st);
void launch_cg_pupdate(double2* p, const double2* s, long n, int nrhs, const double* scal, int gnew_slot,
                       int gold_slot, hipStream_t st);

// ---- multigrid for the normal equations (2d, unsplit P, 9-point box stencils) ----
// One coarsening: fine extents f1 x f2 with dof components per site in layout
// lf, blocks b1 x b2, coarse extents c1 x c2 with M components per site
// ([site][k]); sa: P smoothed (2 x 2 candidate blocks per fine site).
struct NGeom {
  int f1, f2, b1, b2, c1, c2;
  int dof, M, sa;
  Layout lf;
};
size_t normal_orth_lds(const NGeom& g);
// tentative P [Vf][dof][M] from vecs (M fields of layout lf, vstride apart); *err |= 1 on rank deficiency
void launch_normal_orth(double2* Pt, const double2* vecs, const NGeom& g, long vstride, int* err, hipStream_t st);
// (stop: the launch does nothing while *stop != 0)
void launch_normal_prolong(double2* out, const double2* in, const double2* P, const NGeom& g, int nrhs, int accumulate,
                           hipStream_t st, const int* stop = nullptr);
void launch_normal_restrict(double2* out, const double2* in, const double2* P, const NGeom& g, int nrhs,
                            hipStream_t st, const int* stop = nullptr);
// the box stencil Y[V][9][M][M] applied to `in` (layout lay, nrhs fields
// lay.per_rhs() apart) with an epilogue, y = Y in:
enum BoxEpi {
  BOX_APPLY = 0,    // out = y
  BOX_RESID = 1,    // out = b - y
  BOX_SMOOTH0 = 2,  // x = c1 in, out = in - c1 y
  BOX_SMOOTH1 = 3,  // x += c1 in, out = in - c1 y (out != in)
  BOX_POST = 4      // x += c1 in - c2 y
};
struct BoxArgs {
  double2* out = nullptr;
  const double2* in = nullptr;
  const double2* b = nullptr;
  double2* x = nullptr;
  const double2* Y = nullptr;
  int L1 = 0, L2 = 0, M = 0;
  Layout lay{};
  int epi = BOX_APPLY;
  double c1 = 0.0, c2 = 0.0;
  const int* stop = nullptr;  // non-zero *stop: the launch does nothing
};
void launch_box(const BoxArgs& a, int nrhs, hipStream_t st);
void launch_box_dense(double2* A, const double2* Y, int L1, int L2, int M, hipStream_t st);
void launch_probe(double2* e, int c1, int c2, int M, int p1, int p2, int q0, int nq, hipStream_t st);
void launch_galerkin_box_scatter(double2* Y, const double2* z, int c1, int c2, int M, int p1, int p2, int q0, int nq,
                                 hipStream_t st);
void launch_psa_scatter(double2* P, const double2* y, const NGeom& g, int p1, int p2, int q0, int nq,
                        hipStream_t st);
// P as a dense matrix [Vf dof][Vc M] (zeroed before)
void launch_normal_p_dense(double2* out, const double2* P, const NGeom& g, hipStream_t st);
// scal[slot .. slot+2] = Re <a, b>, Im <a, b>, <a, a> (nothing when stop && *stop)
void launch_dot3(const double2* a, const double2* b, long n, RedArgs red, hipStream_t st, const int* stop = nullptr);
// CG steps that run only while *stop == 0.  Direction: p = z + (scal[gnew] /
// scal[gold]) p (p = z when fresh).  Update: alpha = scal[gamma] / scal[qq],
// x += alpha p, r -= alpha q, scal[rr] = |r|^2 (also scal[rr2] when
// rr2 >= 0); its last block sets *stop = (|r|^2 <= tol2) and counts the step
// in *iters.
void launch_cgb_dir(double2* p, const double2* z, long n, const double* scal, int gnew, int gold, int fresh,
                    const int* stop, hipStream_t st);
void launch_cgb_update(double2* x, double2* r, const double2* p, const double2* q, long n, RedArgs red, int gamma,
                       int qq, int rr, int rr2, double tol2, int* stop, int* iters, hipStream_t st);
void launch_mr_step(double2* x, double2* r, const double2* p, const double* scal, int slot, double omega, long n,
                    hipStream_t st);
void launch_smooth_step(double2* x, double2* r, const double2* b, const double2* t, double tau, long n, int first,
                        hipStream_t st, const int* stop = nullptr);
void launch_smooth_post(double2* x, const double2* r, const double2* t, double c1, double c2, long n,
                        hipStream_t st, const int* stop = nullptr);
void launch_axpy3(double2* y, const double2* x, const double2* t, double w, long n, hipStream_t st);
void launch_scale_norm(double2* p, const double2* q, const double* scal, int slot, long n, hipStream_t st);

}  // namespace amg
