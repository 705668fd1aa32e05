// Register-resident Metropolis sweep (reg_walk.h): one wavefront per
// walker, WPB walkers of one instance per workgroup sharing the instance
// tables in LDS.
#include "launch.h"
#include "reg_walk.h"

namespace mvmc {

size_t sweep_reg_lds_bytes(int ne_max, int ns, int M, size_t tsize, int wpb) {
  return reg_table_bytes(ns) + (size_t)wpb * reg_walker_bytes(ne_max, ns, M, tsize);
}

namespace {
template <typename T, int NE_MAX, int WPB, bool TRACE, bool RBM, bool EXCH>
__global__ __launch_bounds__(64 * WPB) void k_sweep_reg(Pools P, const int32_t* __restrict__ wlist,
                                                        int cap, uint64_t seed, TraceRec* trace,
                                                        int64_t trace_cap,
                                                        const uint64_t* __restrict__ trace_base,
                                                        const uint64_t* __restrict__ target,
                                                        int32_t* __restrict__ needs_refresh, int R,
                                                        int kref, int ex64) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wv = sgpr(threadIdx.x >> 6);
  reg_load_tables<WPB>(P, P.inst[P.walker_inst[wlist[blockIdx.x * WPB]]], smem);
  __syncthreads();   // the only workgroup barrier
  reg_walk<T, NE_MAX, WPB, TRACE, RBM, EXCH>(P, sgpr(wlist[blockIdx.x * WPB + wv]), wv, smem, cap,
                                             seed, trace, trace_cap, trace_base, target,
                                             needs_refresh, R, kref, ex64);
}
}  // namespace

template <typename T>
bool launch_sweep_reg(const Pools& P, const int32_t* wlist, int n_groups, int ne_max, int max_ns,
                      int max_M, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
                      const uint64_t* trace_base, const uint64_t* target, int32_t* needs_refresh,
                      int R, int kref, int ex64, hipStream_t s) {
  constexpr int WPB = 4;
  if (n_groups <= 0 || cap <= 0) return true;
  const size_t sh = sweep_reg_lds_bytes(ne_max, max_ns, max_M, sizeof(T), WPB);
#define MVMC_REG_V(NEM, TR, RB, EX)                                                              \
  do {                                                                                           \
    if (sh > 65536)                                                                              \
      (void)hipFuncSetAttribute((const void*)&k_sweep_reg<T, NEM, WPB, TR, RB, EX>,              \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);            \
    hipLaunchKernelGGL((k_sweep_reg<T, NEM, WPB, TR, RB, EX>), dim3(n_groups), dim3(64 * WPB),   \
                       sh, s, P, wlist, cap, seed, trace, trace_cap, trace_base, target,         \
                       needs_refresh, R, kref, ex64);                                            \
    return true;                                                                                 \
  } while (0)
#define MVMC_REG_E(NEM, EX)                                                                      \
  do {                                                                                           \
    if (trace) {                                                                                 \
      if (max_M > 0) MVMC_REG_V(NEM, true, true, EX);                                            \
      MVMC_REG_V(NEM, true, false, EX);                                                          \
    }                                                                                            \
    if (max_M > 0) MVMC_REG_V(NEM, false, true, EX);                                             \
    MVMC_REG_V(NEM, false, false, EX);                                                           \
  } while (0)
#define MVMC_REG(NEM)                                                                            \
  do {                                                                                           \
    if (ex64 > 0) MVMC_REG_E(NEM, true);                                                         \
    MVMC_REG_E(NEM, false);                                                                      \
  } while (0)
  if (ne_max == 32) MVMC_REG(32);
  if (ne_max == 64) MVMC_REG(64);
#undef MVMC_REG_V
#undef MVMC_REG_E
#undef MVMC_REG
  return false;
}

int sweep_reg_class(int ne, size_t tsize) {
  (void)tsize;
  if (ne <= 32) return 32;
  if (ne <= 64) return 64;
  return 0;
}

template bool launch_sweep_reg<double>(const Pools&, const int32_t*, int, int, int, int, int,
                                       uint64_t, TraceRec*, int64_t, const uint64_t*,
                                       const uint64_t*, int32_t*, int, int, int, hipStream_t);
template bool launch_sweep_reg<float>(const Pools&, const int32_t*, int, int, int, int, int,
                                      uint64_t, TraceRec*, int64_t, const uint64_t*,
                                      const uint64_t*, int32_t*, int, int, int, hipStream_t);

}  // namespace mvmc
