// Gauge handle and the reduction scratch every handle owns, shared by the
// library's host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "amg.h"
#include "hostutil.h"
#include "kernels.h"

namespace amg {
namespace host {

// Reduction scratch + scalar / flag storage shared by a handle's kernels.
constexpr int RHS_MAX = 64;
struct Scratch {
  Buf part, ticket, scal, flags;
  double* host = nullptr;  // pinned mirror of a few scalars
  int nslots = 0;
  void init(int nscal, int nflags) {
    part.ensure(sizeof(double) * (size_t)RHS_MAX * (2 * GCR_KMAX + 4) * RED_MAX_BLOCKS);
    ticket.ensure(sizeof(unsigned) * RHS_MAX * TICKETS_PER_RHS);
    HIPC(hipMemset(ticket.p, 0, sizeof(unsigned) * RHS_MAX * TICKETS_PER_RHS));
    scal.ensure(sizeof(double) * nscal);
    HIPC(hipMemset(scal.p, 0, sizeof(double) * nscal));
    flags.ensure(sizeof(int) * nflags);
    HIPC(hipMemset(flags.p, 0, sizeof(int) * nflags));
    if (!host) HIPC(hipHostMalloc((void**)&host, sizeof(double) * RHS_MAX * 4, hipHostMallocDefault));
    nslots = nscal;
  }
  ~Scratch() {
    if (host) (void)hipHostFree(host);
  }
  RedArgs red(int slot, const int* fl = nullptr, double omega = 1.0) const {
    RedArgs r;
    r.part = part.as<double>();
    r.ticket = ticket.as<unsigned>();
    r.scal = scal.as<double>();
    r.slot = slot;
    r.omega = omega;
    r.flags = fl;
    return r;
  }
  // true when flags[off .. off+n) are all set (synchronises the stream)
  bool all_flags(int off, int n, hipStream_t st) {
    int* h = reinterpret_cast<int*>(host + RHS_MAX * 2);
    HIPC(hipMemcpyAsync(h, flags.as<int>() + off, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i)
      if (!h[i]) return false;
    return true;
  }
  // copy n scalars from slot to the pinned mirror and wait for them
  const double* fetch(int slot, int n, hipStream_t st) {
    HIPC(hipMemcpyAsync(host, scal.as<double>() + slot, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return host;
  }
};

}  // namespace host
}  // namespace amg

// ---------------------------------------------------------------------------
// gauge handle
// ---------------------------------------------------------------------------
struct amg_gauge {
  int device = 0;  // HIP device holding the buffers
  int nd = 2;
  int dims[4] = {1, 1, 1, 1};
  long V = 0;
  int nc = 1, ns = 2, dof = 2;
  double mass = 0.0;
  amg::host::Buf U64, U32;
  // 4d: two-row copies of the links when every link is in SU(3) (third row
  // rebuilt in the stencil); empty otherwise
  amg::host::Buf Uc64, Uc32;
  bool compressed = false;
  // internal-layout buffers for amg_apply / amg_apply_internal
  amg::host::Buf tin, tout;
  amg::host::Scratch sc;
  // CGNR work
  amg::host::Buf cg[6];
  template <typename T> const amg::cplx<T>* U() const;
  amg::Layout lay(int prec) const { return amg::Layout{V, dof, prec == AMG_F64 ? 1 : 2}; }
};
template <> inline const double2* amg_gauge::U<double>() const { return U64.as<double2>(); }
template <> inline const float2* amg_gauge::U<float>() const { return U32.as<float2>(); }

namespace amg {
namespace host {

template <typename T>
inline void wilson_apply(const amg_gauge& g, double mass, int dagger, int epi, const cplx<T>* in, cplx<T>* out,
                  const cplx<T>* b, cplx<T>* copy_out, int nrhs, RedArgs red, hipStream_t st) {
  WilsonArgs<T> a;
  a.out = out; a.in = in; a.b = b; a.copy_out = copy_out;
  a.U = g.U<T>();
  if (g.nd == 4 && g.compressed) a.Uc = std::is_same<T, float>::value ? g.Uc32.p : g.Uc64.p;
  a.mass = mass;
  a.L1 = g.dims[0]; a.L2 = g.dims[1]; a.L3 = g.dims[2]; a.L4 = g.dims[3];
  a.nrhs = nrhs;
  a.red = red;
  if (g.nd == 2) launch_wilson2d<T>(a, dagger, epi, st);
  else launch_wilson4d<T>(a, dagger, epi, st);
}

}  // namespace host
}  // namespace amg

