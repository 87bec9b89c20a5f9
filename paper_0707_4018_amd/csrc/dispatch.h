// Kernel dispatch with an optional recorder.
//
// Every solve-path kernel takes its arguments as one trivially copyable
// struct `a0` plus an optional device array `batch` of such structs.  A plain
// launch passes batch = nullptr and runs one problem instance; a batched
// launch runs many instances in one grid, instance = blockIdx.z reading its
// own struct from `batch`.
//
// dispatch() launches immediately, or — while a Recorder is installed on the
// calling thread — appends (kernel, argument bytes, grid, block) to it
// instead.  The batch layer records the same solve sequence once per
// instance and merges the recordings stage by stage into batched launches.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

namespace amg {

struct RecordedLaunch {
  const void* fn = nullptr;
  std::vector<char> args;
  dim3 grid, block;
};

struct Recorder {
  std::vector<RecordedLaunch> ops;
};

Recorder*& current_recorder();

// Kernel timing: an event pair armed for the next launch on this thread.  The
// launch stamps the pair itself (start and end of the kernel's execution),
// so the interval excludes the dispatch gap that events recorded on the
// stream around a launch would include.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming& pending_timing();

template <class A>
inline void dispatch(void (*fn)(A, const A*), const A& a, dim3 grid, dim3 block, hipStream_t st) {
  if (Recorder* rec = current_recorder()) {
    RecordedLaunch r;
    r.fn = reinterpret_cast<const void*>(fn);
    r.args.resize(sizeof(A));
    std::memcpy(r.args.data(), &a, sizeof(A));
    r.grid = grid;
    r.block = block;
    rec->ops.push_back(std::move(r));
    return;
  }
  LaunchTiming& t = pending_timing();
  if (t.start != nullptr) {
    hipExtLaunchKernelGGL(fn, grid, block, 0, st, t.start, t.stop, 0, a, static_cast<const A*>(nullptr));
    t = LaunchTiming{};
    return;
  }
  hipLaunchKernelGGL(fn, grid, block, 0, st, a, static_cast<const A*>(nullptr));
}

// Pick this block's argument struct; blocks past the instance's rhs count
// exit.  The struct is copied field by field from the kernel arguments or
// from the batch table (the copy is split into scalars): a reference that
// could point at either would be a generic pointer, which turns every
// pointer loaded from it into a flat address and every memory access of the
// kernel into a flat instruction (whose waits also wait for scalar loads).
#define AMG_PICK(NAME, ...)                  \
  __VA_ARGS__ NAME;                          \
  if (batch != nullptr) {                    \
    NAME = batch[blockIdx.z];                \
  } else {                                   \
    NAME = a0;                               \
  }
#define AMG_ARGS(...)      \
  AMG_PICK(a, __VA_ARGS__) \
  if ((int)blockIdx.y >= a.nrhs) return;

}  // namespace amg
