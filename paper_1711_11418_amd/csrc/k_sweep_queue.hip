// One persistent launch for the sweeps of a whole ragged batch.
//
// Work items are walkers of the anti-parallel-block tier (one workgroup of
// 256 threads each, M^-1 in LDS, ap_walk.h) and groups of four walkers of
// the register tier (one wavefront each, reg_walk.h).  The host lists them
// in decreasing order of cost (longest first); the grid is as many
// workgroups as fit on the device at once, and every workgroup takes the
// next item from a global counter until the list is empty, so the long
// walkers start first and the short ones fill the tail.  Both tiers
// recompute X^-1 in double inside the launch (at every multiple of
// refresh_every and at a non-finite ratio), so a call makes one launch
// whatever the refresh cadence: the register tier as in its own kernel, an
// anti-parallel-block walker by the workgroup's 16 x 16 Gauss-Jordan
// exchange steps (ap_refresh_tile) between its runs of proposals.
#include <algorithm>
#include <map>
#include <mutex>

#include "ap_refresh.h"
#include "ap_walk.h"
#include "launch.h"
#include "reg_walk.h"

namespace mvmc {

namespace {
constexpr int kQueueThreads = 256;
constexpr int kQueueWpb = kQueueThreads / 64;   // register-tier walkers per item

__global__ void k_queue_reset(int32_t* head) { *head = 0; }

// item >= 0: anti-parallel-block walker `item`; item < 0: register-tier
// group -(item + 1) of `groups` (kQueueWpb global walker ids, -1 padded).
// NEM: register tier of the groups (0 when there are none); NB: register
// blocks of the refresh of the anti-parallel walkers (0 when there are none);
// FULL: both tiers with trace, RBM and exchange code.
template <typename T, int NEM, int NB>
constexpr int queue_waves_per_simd() {
  return NEM > 0 ? 2 : (NB >= 6 ? 2 : (sizeof(T) == 8 ? 2 : 3));
}

template <typename T, int NEM, int NB, bool FULL>
__global__ __launch_bounds__(kQueueThreads)
__attribute__((amdgpu_waves_per_eu(queue_waves_per_simd<T, NEM, NB>()))) void k_sweep_queue(
    Pools P, const int32_t* __restrict__ items, int n_items, const int32_t* __restrict__ groups,
    int32_t* __restrict__ head, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
    const uint64_t* __restrict__ trace_base, const uint64_t* __restrict__ target, int R,
    int ex64) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();   // every thread has the item before thread 0 takes the next
    if (it >= n_items) break;   // uniform
    const int code = items[it];
    if (code >= 0) {
      if constexpr (NB > 0) {
        // runs of proposals up to each multiple of R (or a non-finite
        // ratio), the double-precision refresh between them
        while (ap_walk<T, kQueueThreads, FULL>(P, code, smem, cap, seed, trace, trace_cap,
                                               trace_base, target, nullptr, R, ex64)) {
          __syncthreads();   // the walker's state in memory, for every thread
          ap_refresh_tile<T, NB>(P, code, smem, 0.0, nullptr);
          __syncthreads();
        }
      }
    } else {
      if constexpr (NEM > 0) {
        const int32_t* g = groups + (int64_t)(-code - 1) * kQueueWpb;
        reg_load_tables<kQueueWpb>(P, P.inst[P.walker_inst[g[0]]], smem);
        __syncthreads();
        const int wv = sgpr(threadIdx.x >> 6);
        reg_walk<T, NEM, kQueueWpb, FULL, FULL, FULL>(P, sgpr(g[wv]), wv, smem, cap, seed, trace,
                                                      trace_cap, trace_base, target, nullptr, R,
                                                      1, ex64);
      }
    }
  }
}

template <typename T, int NEM, int NB, bool FULL>
void queue_launch(const Pools& P, const int32_t* items, int n_items, const int32_t* groups,
                  int32_t* head, size_t sh, int n_cu, int cap, uint64_t seed, TraceRec* trace,
                  int64_t trace_cap, const uint64_t* trace_base, const uint64_t* target, int R,
                  int ex64, hipStream_t s) {
  const void* fn = (const void*)&k_sweep_queue<T, NEM, NB, FULL>;
  // workgroups per compute unit for this kernel and LDS size, asked once
  // (the launch itself may be under graph capture)
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> resident;
  static std::map<const void*, size_t> lds_max;   // dynamic-LDS attribute set so far
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (sh > 65536 && sh > lds_max[fn]) {
      (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
      lds_max[fn] = sh;
    }
    auto it = resident.find({fn, sh});
    if (it != resident.end()) {
      per_cu = it->second;
    } else {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kQueueThreads, sh) !=
              hipSuccess ||
          per_cu < 1)
        per_cu = 1;
      resident[{fn, sh}] = per_cu;
    }
  }
  const int64_t grid = std::min<int64_t>(n_items, (int64_t)per_cu * n_cu);
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, head);
  hipLaunchKernelGGL((k_sweep_queue<T, NEM, NB, FULL>), dim3((unsigned)grid), dim3(kQueueThreads),
                     sh, s, P, items, n_items, groups, head, cap, seed, trace, trace_cap,
                     trace_base, target, R, ex64);
}
}  // namespace

int sweep_queue_nb(int max_ne_ap) {
  const int n = max_ne_ap / 2;
  if (n <= 0) return 0;
  if (n <= 4 * kTileT) return 4;
  if (n <= 6 * kTileT) return 6;
  if (n <= 8 * kTileT) return 8;
  return -1;
}

size_t sweep_queue_lds_bytes(int max_ne_reg, int max_ne_ap, int ns, int M, size_t tsize) {
  size_t b = 0;
  if (max_ne_reg > 0) b = sweep_reg_lds_bytes(64, ns, M, tsize, kQueueWpb);
  if (max_ne_ap > 0) {
    b = std::max(b, ap_sweep_layout(max_ne_ap, ns, M, tsize, kQueueThreads / 64).total);
    b = std::max(b, tiled_bytes(max_ne_ap, ns));
  }
  return b;
}

template <typename T>
bool launch_sweep_queue(const Pools& P, const int32_t* items, int n_items, const int32_t* groups,
                        int32_t* head, int max_ne_reg, int max_ne_ap, size_t sh, bool full,
                        int n_cu, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
                        const uint64_t* trace_base, const uint64_t* target, int R, int ex64,
                        hipStream_t s) {
  if (n_items <= 0 || cap <= 0) return true;
  const int nb = sweep_queue_nb(max_ne_ap);
  if (nb < 0 || max_ne_reg > 64 || sh > 160 * 1024) return false;
#define MVMC_Q(NEM, NBV)                                                                        \
  do {                                                                                          \
    if (full)                                                                                   \
      queue_launch<T, NEM, NBV, true>(P, items, n_items, groups, head, sh, n_cu, cap, seed,     \
                                      trace, trace_cap, trace_base, target, R, ex64, s);        \
    else                                                                                        \
      queue_launch<T, NEM, NBV, false>(P, items, n_items, groups, head, sh, n_cu, cap, seed,    \
                                       trace, trace_cap, trace_base, target, R, ex64, s);       \
    return true;                                                                                \
  } while (0)
#define MVMC_QN(NEM)                                                                            \
  do {                                                                                          \
    if (nb == 4) MVMC_Q(NEM, 4);                                                                \
    if (nb == 6) MVMC_Q(NEM, 6);                                                                \
    if (nb == 8) MVMC_Q(NEM, 8);                                                                \
  } while (0)
  if (max_ne_reg > 0) {
    if (nb == 0) MVMC_Q(64, 0);
    MVMC_QN(64);
  } else {
    MVMC_QN(0);
  }
#undef MVMC_Q
#undef MVMC_QN
  return false;
}

template bool launch_sweep_queue<double>(const Pools&, const int32_t*, int, const int32_t*,
                                         int32_t*, int, int, size_t, bool, int, int, uint64_t,
                                         TraceRec*, int64_t, const uint64_t*, const uint64_t*,
                                         int, int, hipStream_t);
template bool launch_sweep_queue<float>(const Pools&, const int32_t*, int, const int32_t*,
                                        int32_t*, int, int, size_t, bool, int, int, uint64_t,
                                        TraceRec*, int64_t, const uint64_t*, const uint64_t*,
                                        int, int, hipStream_t);

}  // namespace mvmc
