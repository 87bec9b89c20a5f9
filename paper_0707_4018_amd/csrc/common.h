// Device-side helpers shared by the gfx950 kernels of libamg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amg {

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
template <typename T> __device__ __forceinline__ cplx<T> ldp(const double2* p, long i) { const double2 z = p[i]; return mk<T>((T)z.x, (T)z.y); }
template <typename T> __device__ __forceinline__ cplx<T> ldp(const float2* p, long i) { const float2 z = p[i]; return mk<T>((T)z.x, (T)z.y); }
template <typename T> __device__ __forceinline__ cplx<T> ldp(const bf16x2* p, long i) { const bf16x2 z = p[i]; return mk<T>((T)bf2f(z.x), (T)bf2f(z.y)); }

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
// last block to arrive (atomic ticket per rhs) sums the partials in block
// order and returns true with the totals in `tot` (valid in all threads).
// The sum order is fixed, so results do not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
constexpr int RED_WAVES = RED_THREADS / 64;

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[RED_WAVES]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_WAVES; ++w) s += sh[k][w];
    v[k] = s;
  }
  __syncthreads();
}

template <int NV>
__device__ bool grid_reduce(double (&v)[NV], double* part, unsigned* ticket, int rhs,
                            double (&tot)[NV]) {
  __shared__ double sh[NV][RED_WAVES];
  __shared__ int is_last;
  const int nblk = gridDim.x;
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) part[((long)rhs * NV + k) * nblk + blockIdx.x] = v[k];
    __threadfence();
    const unsigned t = atomicAdd(&ticket[rhs], 1u);
    is_last = (t == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!is_last) return false;
  // acquire: every block released its partials (fence) before taking a
  // ticket, and this fence invalidates the local caches, so plain loads see
  // them; plain loads can all be in flight at once, unlike coherent ones
  __threadfence();
  double s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) s[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] += part[((long)rhs * NV + k) * nblk + b];
  }
  block_sum<NV>(s, sh);
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = s[k];
  if (threadIdx.x == 0)
    __hip_atomic_store(&ticket[rhs], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Scalars and flags of a solver live in one device array of doubles.
// A right-hand side whose `skip` flag is non-zero is left untouched.
__device__ __forceinline__ bool skip_rhs(const int* flags, int rhs) {
  return flags != nullptr && flags[rhs] != 0;
}

}  // namespace amg
