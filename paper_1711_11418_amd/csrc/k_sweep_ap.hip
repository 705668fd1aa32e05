// Metropolis sweep on the anti-parallel block alone (ap_walk.h): one
// workgroup per walker keeps only M^-1 (n x n, n = N_e/2) in LDS for the
// whole launch and stops at every multiple of refresh_every and at a
// non-finite ratio for the refresh kernel.  Proposal, correlators, trace,
// refresh cadence and non-finite guard are those of k_sweep.hip.
#include "ap_walk.h"
#include "launch.h"

namespace mvmc {

size_t sweep_ap_lds_bytes(int ne, int ns, int M, size_t tsize, int nthreads) {
  return ap_sweep_layout(ne, ns, M, tsize, nthreads / 64).total;
}

namespace {
// Register budget of four waves per SIMD in single precision, three in
// double (four would spill the double variants).
// FULL = false: the walkers of the launch have no RBM factor, no trace and
// no exchange updates.
template <typename T, int NT, bool FULL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void k_sweep_ap(Pools P, const int32_t* __restrict__ wlist, int cap, uint64_t seed,
                TraceRec* trace, int64_t trace_cap, const uint64_t* __restrict__ trace_base,
                const uint64_t* __restrict__ target, int32_t* __restrict__ needs_refresh, int R,
                int ex64) {
  extern __shared__ __align__(16) unsigned char smem[];
  (void)ap_walk<T, NT, FULL>(P, wlist[blockIdx.x], smem, cap, seed, trace, trace_cap, trace_base,
                             target, needs_refresh, R, ex64);
}
}  // namespace

template <typename T>
void launch_sweep_ap(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                     int max_ne, int max_ns, int max_M, int nthreads, TraceRec* trace,
                     int64_t trace_cap, const uint64_t* trace_base, const uint64_t* target,
                     int32_t* needs_refresh, int R, int ex64, hipStream_t s) {
  if (n <= 0 || cap <= 0) return;
  const size_t sh = ap_sweep_layout(max_ne, max_ns, max_M, sizeof(T), nthreads / 64).total;
  const bool full = trace != nullptr || ex64 > 0 || max_M > 0;
#define MVMC_AP_LAUNCH(NTV, FV)                                                                  \
  do {                                                                                           \
    if (sh > 65536)                                                                              \
      (void)hipFuncSetAttribute((const void*)&k_sweep_ap<T, NTV, FV>,                            \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);            \
    hipLaunchKernelGGL((k_sweep_ap<T, NTV, FV>), dim3(n), dim3(NTV), sh, s, P, wlist, cap, seed, \
                       trace, trace_cap, trace_base, target, needs_refresh, R, ex64);            \
  } while (0)
  if (full) {
    if (nthreads == 64) MVMC_AP_LAUNCH(64, true);
    else if (nthreads == 128) MVMC_AP_LAUNCH(128, true);
    else MVMC_AP_LAUNCH(256, true);
  } else {
    if (nthreads == 64) MVMC_AP_LAUNCH(64, false);
    else if (nthreads == 128) MVMC_AP_LAUNCH(128, false);
    else MVMC_AP_LAUNCH(256, false);
  }
#undef MVMC_AP_LAUNCH
}

template void launch_sweep_ap<double>(const Pools&, const int32_t*, int, int, uint64_t, int, int,
                                      int, int, TraceRec*, int64_t, const uint64_t*,
                                      const uint64_t*, int32_t*, int, int, hipStream_t);
template void launch_sweep_ap<float>(const Pools&, const int32_t*, int, int, uint64_t, int, int,
                                     int, int, TraceRec*, int64_t, const uint64_t*,
                                     const uint64_t*, int32_t*, int, int, hipStream_t);

}  // namespace mvmc
