// Host stand-in for the HIP device environment, for the CPU emulation tests
// of the library's kernels.  Every lane of a workgroup is a user-level fiber
// (ucontext); a barrier is a yield to a round-robin scheduler that resumes
// each lane in turn, so all lanes reach every barrier before any passes it.
// emu_launch runs the workgroups one after the other; emu_launch_grid runs
// them at the same time, one host thread each (for kernels that wait on each
// other through device atomics; a wave's sleep yields the host thread).
// Workgroup state (fibers, shared memory, thread and block indices) is per
// host thread.  Wavefront shuffles, DPP row operations and readlane are
// emulated through a slot per lane and two barriers (all lanes execute them
// together, as on the device).  Test infrastructure only: nothing in the
// library uses it.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
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
#define __shared__ static thread_local
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_fence(a, b) std::atomic_thread_fence(std::memory_order_seq_cst)

struct emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
inline thread_local emu_dim3 threadIdx, blockIdx;
inline emu_dim3 gridDim, blockDim;

// fiber scheduler
inline thread_local ucontext_t emu_main_ctx;
inline thread_local std::vector<ucontext_t> emu_lane_ctx;
inline thread_local int emu_cur = 0;
inline void emu_yield() { swapcontext(&emu_lane_ctx[emu_cur], &emu_main_ctx); }
// Barriers count arrivals: a lane waits (yielding) until every lane of its
// workgroup (__syncthreads) or of its wave (wave barrier) has arrived.
inline thread_local unsigned emu_blk_count = 0, emu_blk_gen = 0;
inline thread_local unsigned emu_wave_count[16], emu_wave_gen[16];
inline void __syncthreads() {
  const unsigned g = emu_blk_gen;
  if (++emu_blk_count == blockDim.x) {
    emu_blk_count = 0;
    ++emu_blk_gen;
  } else {
    while (emu_blk_gen == g) emu_yield();
  }
}
inline void __builtin_amdgcn_wave_barrier() {
  const int w = threadIdx.x >> 6;
  const unsigned width = std::min(64u, blockDim.x - 64u * w);
  const unsigned g = emu_wave_gen[w];
  if (++emu_wave_count[w] == width) {
    emu_wave_count[w] = 0;
    ++emu_wave_gen[w];
  } else {
    while (emu_wave_gen[w] == g) emu_yield();
  }
}

// one exchange slot per lane; a value is published, then read from lane src
inline thread_local long long emu_slot[1024];
inline void __builtin_amdgcn_wave_barrier();
inline long long emu_exchange(long long v, int src_lane_in_wave, bool valid, long long fallback) {
  const int l = threadIdx.x;
  emu_slot[l] = v;
  __builtin_amdgcn_wave_barrier();
  const long long r = valid ? emu_slot[l - (l & 63) + src_lane_in_wave] : fallback;
  __builtin_amdgcn_wave_barrier();
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
inline unsigned atomicAdd(unsigned* p, unsigned v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicExch(unsigned* p, unsigned v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
inline int atomicExch(int* p, int v) { return __atomic_exchange_n(p, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
  unsigned long long o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (o < v && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return o;
}
#define __HIP_MEMORY_SCOPE_AGENT 0
template <class T>
inline T __hip_atomic_load(const T* p, int, int) {
  T r;
  __atomic_load(const_cast<T*>(p), &r, __ATOMIC_SEQ_CST);
  return r;
}
template <class T, class U>
inline void __hip_atomic_store(T* p, U v, int, int) {
  T x = (T)v;
  __atomic_store(p, &x, __ATOMIC_SEQ_CST);
}
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::yield(); }
inline int __shfl(int v, int src, int w = 64) { return (int)emu_exchange(v, src & 63, true, v); }
inline double __shfl(double v, int src, int w = 64) {
  return __longlong_as_double(emu_exchange(__double_as_longlong(v), src & 63, true, __double_as_longlong(v)));
}
inline double __shfl_xor(double v, int mask, int w = 64) {
  const int lane = threadIdx.x & 63;
  return __longlong_as_double(emu_exchange(__double_as_longlong(v), lane ^ mask, true, __double_as_longlong(v)));
}
// raw buffer accesses (device-scope coherent loads and stores of 8 bytes)
struct __amdgpu_buffer_rsrc_t {
  char* base;
};
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short, int, int) { return {(char*)p}; }
struct emu_v2u {
  unsigned x, y;
};
inline emu_v2u __builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t r, int off, int soff, int) {
  emu_v2u v;
  __atomic_load((emu_v2u*)(r.base + off + soff), &v, __ATOMIC_SEQ_CST);
  return v;
}
inline void __builtin_amdgcn_raw_buffer_store_b64(emu_v2u v, __amdgpu_buffer_rsrc_t r, int off, int soff, int) {
  __atomic_store((emu_v2u*)(r.base + off + soff), &v, __ATOMIC_SEQ_CST);
}
// dynamic shared memory of the current workgroup (sized by the launch)
inline thread_local std::vector<double> emu_dyn_lds;
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(emu_dyn_lds.data());
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
// Workgroups b0, b0 + step, ... < blocks on the calling host thread.
template <class F>
void emu_run_blocks(int b0, int step, int blocks, int threads, F& f, size_t dyn_lds_bytes) {
  constexpr size_t kStack = 512 * 1024;
  // fiber stacks left uninitialised: pages are committed only when used
  std::vector<std::unique_ptr<char[]>> stacks(threads);
  for (auto& st : stacks) st.reset(new char[kStack]);
  std::vector<char> done_store(threads);
  bool* done = (bool*)done_store.data();
  emu_task<F> task{&f, done};
  const uintptr_t p = (uintptr_t)&task;
  emu_dyn_lds.assign(dyn_lds_bytes / 8 + 1, 0.0);
  for (int b = b0; b < blocks; b += step) {
    blockIdx.x = b;
    emu_blk_count = emu_blk_gen = 0;
    for (int w = 0; w < 16; ++w) emu_wave_count[w] = emu_wave_gen[w] = 0;
    emu_lane_ctx.assign(threads, ucontext_t{});
    for (int t = 0; t < threads; ++t) {
      done[t] = false;
      getcontext(&emu_lane_ctx[t]);
      emu_lane_ctx[t].uc_stack.ss_sp = stacks[t].get();
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

template <class F>
void emu_launch(int blocks, int threads, F f, size_t dyn_lds_bytes = 0) {
  gridDim.x = blocks;
  blockDim.x = threads;
  emu_run_blocks(0, 1, blocks, threads, f, dyn_lds_bytes);
}

// All workgroups resident at once, as a cooperative launch: one host thread
// per workgroup.
template <class F>
void emu_launch_grid(int blocks, int threads, F f, size_t dyn_lds_bytes = 0) {
  gridDim.x = blocks;
  blockDim.x = threads;
  std::vector<std::thread> th;
  for (int b = 0; b < blocks; ++b)
    th.emplace_back([&, b]() { emu_run_blocks(b, blocks, blocks, threads, f, dyn_lds_bytes); });
  for (auto& t : th) t.join();
}
