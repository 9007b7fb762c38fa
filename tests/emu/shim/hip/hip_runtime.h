// Host stand-in for the HIP device environment, for the CPU emulation test
// of the strip-layout sweep kernels.  Every lane of a workgroup is a
// user-level fiber (ucontext); a barrier is a yield to a round-robin
// scheduler that resumes each lane in turn, so all lanes reach every barrier
// before any passes it.  Workgroups run one after the other.  Wavefront
// shuffles, DPP row operations and readlane are emulated through a slot per
// lane and two barriers (all lanes execute them together, as on the
// device).  Test infrastructure only: nothing in the library uses it.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <ucontext.h>
#include <vector>
using std::max;
using std::min;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __restrict__
#define __align__(x)
#define __shared__ static
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_fence(a, b) std::atomic_thread_fence(std::memory_order_seq_cst)

struct emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
inline emu_dim3 threadIdx, blockIdx, gridDim, blockDim;

// fiber scheduler
inline ucontext_t emu_main_ctx;
inline std::vector<ucontext_t> emu_lane_ctx;
inline int emu_cur = 0;
inline void __syncthreads() { swapcontext(&emu_lane_ctx[emu_cur], &emu_main_ctx); }
inline void __builtin_amdgcn_wave_barrier() { __syncthreads(); }

// one exchange slot per lane; a value is published, then read from lane src
inline long long emu_slot[1024];
inline long long emu_exchange(long long v, int src_lane_in_wave, bool valid, long long fallback) {
  const int l = threadIdx.x;
  emu_slot[l] = v;
  __syncthreads();
  const long long r = valid ? emu_slot[l - (l & 63) + src_lane_in_wave] : fallback;
  __syncthreads();
  return r;
}
inline long long __double_as_longlong(double d) {
  long long x;
  memcpy(&x, &d, 8);
  return x;
}
inline double __longlong_as_double(long long x) {
  double d;
  memcpy(&d, &x, 8);
  return d;
}
inline double __shfl_up(double v, int d, int w = 64) {
  const int lane = threadIdx.x & 63;
  return __longlong_as_double(emu_exchange(__double_as_longlong(v), lane - d, lane - d >= 0, __double_as_longlong(v)));
}
inline double __shfl_down(double v, int d, int w = 64) {
  const int lane = threadIdx.x & 63;
  return __longlong_as_double(emu_exchange(__double_as_longlong(v), lane + d, lane + d < w, __double_as_longlong(v)));
}
// DPP controls used by the kernels: row_shl:1-15, row_shr:1-15,
// row_bcast:15, row_bcast:31.  emu_dpp_source gives the source lane and
// whether the lane is written (row in row_mask, source in range).
inline bool emu_dpp_source(int ctrl, int row_mask, int* sl) {
  const int lane = threadIdx.x & 63, inrow = lane & 15, row = lane >> 4;
  bool ok = true;
  *sl = lane;
  if (ctrl >= 0x101 && ctrl <= 0x10f) {
    ok = inrow + (ctrl - 0x100) < 16;
    *sl = lane + (ctrl - 0x100);
  } else if (ctrl >= 0x111 && ctrl <= 0x11f) {
    ok = inrow >= ctrl - 0x110;
    *sl = lane - (ctrl - 0x110);
  } else if (ctrl == 0x142) {
    ok = row >= 1;
    *sl = 16 * row - 1;
  } else if (ctrl == 0x143) {
    ok = row >= 2;
    *sl = 31;
  } else {
    fprintf(stderr, "dpp control %#x is not emulated\n", ctrl);
    abort();
  }
  if (!((row_mask >> row) & 1)) ok = false;
  if (!ok) *sl = lane;
  return ok;
}
// Lanes not written keep `old` (bound_ctrl off).
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  int sl;
  const bool ok = emu_dpp_source(ctrl, row_mask, &sl);
  if (bound_ctrl) {
    fprintf(stderr, "update_dpp with bound_ctrl is not emulated\n");
    abort();
  }
  return (int)emu_exchange(src, sl, ok, old);
}
// All rows written (row_mask 0xf); lanes whose source is out of range read 0
// (bound_ctrl on).
inline int __builtin_amdgcn_mov_dpp(int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  if (row_mask != 0xf || !bound_ctrl) {
    fprintf(stderr, "mov_dpp is emulated for row_mask 0xf with bound_ctrl only\n");
    abort();
  }
  int sl;
  const bool ok = emu_dpp_source(ctrl, row_mask, &sl);
  return (int)emu_exchange(src, sl, ok, 0);
}
inline int __builtin_amdgcn_readlane(int v, int l) { return (int)emu_exchange(v, l, true, 0); }
inline int atomicAdd(int* p, int v) { return reinterpret_cast<std::atomic<int>*>(p)->fetch_add(v); }
struct double2 {
  double x, y;
};
inline double2 make_double2(double a, double b) { return {a, b}; }

// Run `blocks` workgroups of `threads` lanes, one after the other.
template <class F>
struct emu_task {
  F* f;
  bool* done;
};
template <class F>
void emu_entry(unsigned lo, unsigned hi) {
  const uintptr_t p = ((uintptr_t)hi << 32) | lo;
  emu_task<F>* t = (emu_task<F>*)p;
  (*t->f)();
  t->done[emu_cur] = true;
}
template <class F>
void emu_launch(int blocks, int threads, F f) {
  gridDim.x = blocks;
  blockDim.x = threads;
  constexpr size_t kStack = 512 * 1024;
  std::vector<std::vector<char>> stacks(threads, std::vector<char>(kStack));
  std::vector<char> done_store(threads);
  bool* done = (bool*)done_store.data();
  emu_task<F> task{&f, done};
  const uintptr_t p = (uintptr_t)&task;
  for (int b = 0; b < blocks; ++b) {
    blockIdx.x = b;
    emu_lane_ctx.assign(threads, ucontext_t{});
    for (int t = 0; t < threads; ++t) {
      done[t] = false;
      getcontext(&emu_lane_ctx[t]);
      emu_lane_ctx[t].uc_stack.ss_sp = stacks[t].data();
      emu_lane_ctx[t].uc_stack.ss_size = kStack;
      emu_lane_ctx[t].uc_link = &emu_main_ctx;
      makecontext(&emu_lane_ctx[t], (void (*)())emu_entry<F>, 2, (unsigned)(p & 0xffffffffu), (unsigned)(p >> 32));
    }
    for (bool all = false; !all;) {
      all = true;
      for (int t = 0; t < threads; ++t) {
        if (done[t]) continue;
        emu_cur = t;
        threadIdx.x = t;
        swapcontext(&emu_main_ctx, &emu_lane_ctx[t]);
        all = all && done[t];
      }
    }
  }
}
