// Device-side helpers shared by the gfx950 kernels of libamg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

// Global-memory views of pointers.  A pointer read out of an argument struct
// is generic, and the compiler then emits flat instructions for it (which
// also count against the scalar/LDS wait counter, so a wait for an argument
// or an LDS value waits for every load in flight).  Kernels access their
// fields through these views instead.
// (The host pass only type-checks device code: there the views are plain.)
#if defined(__HIP_DEVICE_COMPILE__)
#define AMG_GLOBAL __attribute__((address_space(1)))
#else
#define AMG_GLOBAL
#endif
template <typename T> using gptr = AMG_GLOBAL T*;
template <typename T> __device__ __forceinline__ gptr<const T> gl(const T* p) { return (gptr<const T>)p; }
template <typename T> __device__ __forceinline__ gptr<T> gl(T* p) { return (gptr<T>)p; }

// Element i (0 <= i < 4) of a four-entry array, by selects.  Argument
// structs are copied into registers at kernel entry; an array member indexed
// by a run-time value would keep the whole copy in scratch memory, so loops
// over dimensions run to 4 with a guard and read arrays through this.
template <typename T> __device__ __forceinline__ T at4(const T (&a)[4], int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : a[3]));
}

// ---------------------------------------------------------------------------
// complex arithmetic on float2 / double2
// ---------------------------------------------------------------------------
template <typename T> struct C2;
template <> struct C2<double> { using t = double2; };
template <> struct C2<float> { using t = float2; };
template <typename T> using cplx = typename C2<T>::t;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
  cplx<T> z; z.x = re; z.y = im; return z;
}
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cscale(T s, cplx<T> a) { return mk<T>(s * a.x, s * a.y); }
// a * b
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cplx<T> cjmul(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc += a * b
template <typename T> __device__ __forceinline__ void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
template <typename T> __device__ __forceinline__ void cjfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}
// i * a
template <typename T> __device__ __forceinline__ cplx<T> ctimesi(cplx<T> a) { return mk<T>(-a.y, a.x); }

// ---------------------------------------------------------------------------
// bfloat16 storage (round to nearest even), used for the prolongator
// ---------------------------------------------------------------------------
struct bf16x2 { uint16_t x, y; };

__host__ __device__ __forceinline__ uint16_t f2bf(float f) {
  union { float f; uint32_t u; } v; v.f = f;
  uint32_t u = v.u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf2f(uint16_t h) {
  union { float f; uint32_t u; } v; v.u = ((uint32_t)h) << 16; return v.f;
}

// load an element of P in any storage and return it in compute precision T
template <typename T> __device__ __forceinline__ cplx<T> pval(double2 z) { return mk<T>((T)z.x, (T)z.y); }
template <typename T> __device__ __forceinline__ cplx<T> pval(float2 z) { return mk<T>((T)z.x, (T)z.y); }
template <typename T> __device__ __forceinline__ cplx<T> pval(bf16x2 z) { return mk<T>((T)bf2f(z.x), (T)bf2f(z.y)); }
// element i of P (any storage kind, generic or global pointer) in precision T
template <typename T, typename Ptr> __device__ __forceinline__ cplx<T> ldp(Ptr p, long i) { return pval<T>(p[i]); }
// 16 bytes of P (4 BF16, 2 FP32 or 1 FP64 complex entries) from a 16-byte aligned address
template <typename T, typename PT, typename Ptr>
__device__ __forceinline__ void ldp16(Ptr p, cplx<T> (&out)[16 / sizeof(PT)]) {
  const uint4 v = *reinterpret_cast<const AMG_GLOBAL uint4*>(p);
  PT t[16 / sizeof(PT)];
  __builtin_memcpy(t, &v, 16);
#pragma unroll
  for (int n = 0; n < (int)(16 / sizeof(PT)); ++n) out[n] = pval<T>(t[n]);
}

// ---------------------------------------------------------------------------
// Field layout.  A level field of V sites with `dof` complex components per
// site is stored per right-hand side as units of W complex numbers:
//   offset(site, c) = ((c / W) * V + site) * W + c % W      (complex units)
// W = 1 gives structure-of-arrays planes, W = dof array-of-structures.  The
// fine level uses W = 1 in FP64 (16-byte double2 per lane) and W = 2 in FP32
// (16-byte float4 per lane); coarse levels use W = dof.
// ---------------------------------------------------------------------------
struct Layout {
  long V;
  int dof;
  int W;
  __host__ __device__ __forceinline__ long off(long site, int c) const {
    return ((long)(c / W) * V + site) * W + (c % W);
  }
  __host__ __device__ __forceinline__ long per_rhs() const { return V * dof; }
};

// ---------------------------------------------------------------------------
// Deterministic block + grid reductions of NV doubles per right-hand side.
// Every block writes its partial sums to part[(rhs*NV + k)*nblk + block]; the
// last block to arrive (atomic tickets per rhs) sums the partials in a fixed
// order and returns true with the totals in `tot` (valid in all threads), so
// results do not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
constexpr int RED_WAVES = RED_THREADS / 64;

// Sum over the 64 lanes of a wave with DPP row operations (no trip through
// the LDS crossbar, unlike shuffles): shift-right by 1, 2, 4, 8 within each
// row of 16 lanes leaves the row's sum in its lane 15; broadcasting lane 15
// into the next row, then lane 31 into rows 2 and 3, leaves the total in lane
// 63, which is read into every lane.  Lanes whose DPP source lies outside the
// row add zero.  The order of the additions is fixed.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Publication without a release fence: on this chip each XCD has its own L2,
// and an agent-scope release fence (__threadfence) writes back the whole L2
// of the XCD — for a launch of ~1000 blocks that alone costs tens of
// microseconds.  Only the partial sums have to cross XCDs inside the launch
// (everything else is read by later launches), so each block stores its
// partials with agent-scope atomic stores (written through to the memory
// side), waits until those stores are complete, and only then takes a ticket;
// the last block reads the partials with agent-scope atomic loads, which do
// not hit stale lines of its own L2.  The loads come after the ticket that
// proves every store complete.
// Wait until this thread's earlier memory operations are complete (the
// compiler may not move memory operations across it either).
__device__ __forceinline__ void wait_stores_complete() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Arrival counters: a launch of up to RED_ONE_LEVEL blocks takes tickets of
// one counter (one atomic round trip); a larger one takes two levels — a
// ticket of the block's group of RED_GROUP blocks, then the last of each group
// a ticket of the launch — so no counter sees more than RED_GROUP atomics
// (~1000 atomics on one address serialise for ~8 us).  Each counter has a
// 64-byte line of its own.
constexpr int RED_ONE_LEVEL = 64;
constexpr int RED_GROUP = 32;
constexpr int TICKET_PAD = 16;
constexpr int RED_BLOCKS_LIMIT = 1024;
constexpr int TICKETS_PER_RHS = (1 + RED_BLOCKS_LIMIT / RED_GROUP) * TICKET_PAD;

__device__ __forceinline__ bool take_ticket(unsigned* t, unsigned n) {
  if (__hip_atomic_fetch_add(t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != n - 1) return false;
  __hip_atomic_store(t, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // all n arrived: reset for the next launch
  return true;
}
// Called by one thread per block after its partials are complete; true in
// the block that arrives last in the launch (for right-hand side rhs).
__device__ __forceinline__ bool last_block(unsigned* ticket, int rhs) {
  unsigned* tk = ticket + (long)rhs * TICKETS_PER_RHS;
  const int nblk = gridDim.x;
  if (nblk <= RED_ONE_LEVEL) return take_ticket(tk, (unsigned)nblk);
  const int grp = blockIdx.x / RED_GROUP;
  const int ngrp = (nblk + RED_GROUP - 1) / RED_GROUP;
  const int gsize = (nblk - grp * RED_GROUP < RED_GROUP) ? nblk - grp * RED_GROUP : RED_GROUP;
  if (!take_ticket(tk + (1 + grp) * TICKET_PAD, (unsigned)gsize)) return false;
  return take_ticket(tk, (unsigned)ngrp);
}

// Quantities z0 <= q < z1 are known to be zero in every block (unused slots
// of a template-sized set): they are neither summed nor published, and their
// totals are zero.
template <int NV>
__device__ bool grid_reduce(double (&v)[NV], double* part, unsigned* ticket, int rhs,
                            double (&tot)[NV], int z0 = NV, int z1 = NV) {
  static_assert(NV <= RED_THREADS, "one thread per quantity at least");
  __shared__ double sh[NV][RED_WAVES];
  __shared__ int is_last;
  const int nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k >= z0 && k < z1) continue;  // uniform
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  // thread q publishes the block's sum of quantity q
  if (threadIdx.x < NV && !(threadIdx.x >= z0 && threadIdx.x < z1)) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_WAVES; ++w) s += sh[threadIdx.x][w];
    __hip_atomic_store(&part[((long)rhs * NV + threadIdx.x) * nblk + blockIdx.x], s, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    wait_stores_complete();
  }
  __syncthreads();
  if (threadIdx.x == 0) is_last = last_block(ticket, rhs);
  __syncthreads();
  if (!is_last) return false;
  // thread t sums quantity q = t mod NV over every G-th block from
  // g = t / NV (G = blockDim / NV groups: few loads per thread, all
  // independent), then one wave per quantity adds the G group sums
  __shared__ double shg[RED_THREADS];
  constexpr int G = RED_THREADS / NV;
  const int q = threadIdx.x % NV, g = threadIdx.x / NV;
  if (g < G && !(q >= z0 && q < z1)) {
    double s = 0.0;
    double* pq = part + ((long)rhs * NV + q) * nblk;
    for (int b0 = g; b0 < nblk; b0 += 16 * G) {
      double v[16];  // up to 16 loads in flight, then the adds in block order
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int b = b0 + u * G;
        v[u] = (b < nblk) ? __hip_atomic_load(pq + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
    shg[g * NV + q] = s;
  }
  __syncthreads();
  __shared__ double shtot[NV];
  for (int qq = wave; qq < NV; qq += RED_WAVES) {  // one wave per quantity
    if (qq >= z0 && qq < z1) {
      if (lane == 0) shtot[qq] = 0.0;
      continue;
    }
    double s = 0.0;
    for (int gg = lane; gg < G; gg += 64) s += shg[gg * NV + qq];
    s = wave_sum(s);
    if (lane == 0) shtot[qq] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = shtot[k];
  return true;
}

// Largest grid whose per-block partial sums sum_partials accepts.
constexpr int RED_MAX_PART_BLOCKS = 1024;

// Per-block sums only: thread q < NV stores the block's sum of quantity q to
// part[(rhs NV + q) gridDim.x + block] with a plain store; the kernel that
// consumes them runs after this launch, which makes them visible.
template <int NV>
__device__ void block_partials(double (&v)[NV], double* part, int rhs) {
  __shared__ double sh[NV][RED_WAVES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_WAVES; ++w) s += sh[threadIdx.x][w];
    gl(part)[((long)rhs * NV + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// Totals of the NV partial sums of nblk blocks written by block_partials
// (every block of the consuming kernel computes them, in the same fixed
// order, so all get identical values).  Returns them in every thread.
template <int NV>
__device__ void sum_partials(const double* part, int nblk, int rhs, double (&tot)[NV]) {
  __shared__ double sh[NV][RED_WAVES];
  __shared__ double shtot[NV];
  constexpr int U = (RED_MAX_PART_BLOCKS + RED_THREADS - 1) / RED_THREADS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  gptr<const double> p = gl(part);
  // all of this thread's loads first, then the adds in block order
  double v[NV][U];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = threadIdx.x + u * RED_THREADS;
      v[k][u] = (b < nblk) ? p[((long)rhs * NV + k) * nblk + b] : 0.0;
    }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[k][u];
    s = wave_sum(s);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_WAVES; ++w) s += sh[threadIdx.x][w];
    shtot[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = shtot[k];
}

// Scalars and flags of a solver live in one device array of doubles.
// A right-hand side whose `skip` flag is non-zero is left untouched.
__device__ __forceinline__ bool skip_rhs(const int* flags, int rhs) {
  return flags != nullptr && gl(flags)[rhs] != 0;
}

}  // namespace amg
