// Double-precision recomputation of walkers through the anti-parallel block
// of X (Eq. AP-Pf; ap_refresh.h): one wavefront per walker for N_e <= 64,
// two (the tableau split by columns) for N_e <= 128, one 16 x 16 workgroup
// per walker for N_e <= 256.
#include "ap_refresh.h"
#include "launch.h"

namespace mvmc {

namespace {
constexpr int kApWpb = 4;   // walkers (wavefronts) per workgroup of the one-wave kernel

template <typename T, int NS>
__global__ __launch_bounds__(64 * kApWpb, 2) void k_refresh_ap(Pools P,
                                                             const int32_t* __restrict__ wlist,
                                                             int n, int max_sites, int wld,
                                                             double sing_tol,
                                                             int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wv = threadIdx.x >> 6;
  const int idx = blockIdx.x * kApWpb + wv;
  if (idx >= n) return;
  unsigned char* q = smem + (size_t)wv * (ap_walker_bytes(NS, max_sites) + ap_minv_bytes<T>(wld));
  ap_refresh_wave<T, NS>(P, wlist[idx], q, max_sites, wld, sing_tol, flags);
}

// 32 < n <= 64: two wavefronts per walker.
template <typename T>
__global__ __launch_bounds__(kPairThreads) void k_refresh_ap_pair(
    Pools P, const int32_t* __restrict__ wlist, double sing_tol, int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  ap_refresh_pair<T>(P, wlist[blockIdx.x], smem, sing_tol, flags, flags == nullptr);
}

// 64 < n <= 128: one workgroup of 16 x 16 threads per walker.
template <typename T, int NB>
__global__ __launch_bounds__(kTileThreads, 2) void k_refresh_ap_tiled(
    Pools P, const int32_t* __restrict__ wlist, double sing_tol, int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  ap_refresh_tile<T, NB>(P, wlist[blockIdx.x], smem, sing_tol, flags);
}
}  // namespace

int refresh_ap_route(int max_ne, int max_ns) {
  if (max_ne <= 128 &&
      (ap_walker_bytes(64, max_ns) + ap_minv_bytes<double>(max_ne / 2 + 1)) * kApWpb <= 152 * 1024)
    return 1;
  if (max_ne <= 2 * kTileT * 8 && tiled_bytes(max_ne, max_ns) <= 64 * 1024) return 2;
  return 0;
}

template <typename T>
void launch_refresh_ap(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                       int route, double sing_tol, int32_t* flags, hipStream_t s) {
  if (n <= 0) return;
  if (route == 2) {   // 64 < n_sigma <= 128: the tiled kernel, one workgroup per walker
    hipLaunchKernelGGL((k_refresh_ap_tiled<T, 8>), dim3(n), dim3(kTileThreads),
                       tiled_bytes(max_ne, max_ns), s, P, wlist, sing_tol, flags);
    return;
  }
  const int blocks = (n + kApWpb - 1) / kApWpb;
  const int wld = max_ne / 2 + 1;
  if (max_ne <= 64) {
    const size_t sh = (ap_walker_bytes(32, max_ns) + ap_minv_bytes<T>(wld)) * kApWpb;
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)&k_refresh_ap<T, 32>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh_ap<T, 32>), dim3(blocks), dim3(64 * kApWpb), sh, s, P, wlist, n,
                       max_ns, wld, sing_tol, flags);
  } else {
    const size_t sh = pair_bytes<T>(max_ne, max_ns);
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)&k_refresh_ap_pair<T>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh_ap_pair<T>), dim3(n), dim3(kPairThreads), sh, s, P, wlist,
                       sing_tol, flags);
  }
}

template void launch_refresh_ap<double>(const Pools&, const int32_t*, int, int, int, int, double,
                                        int32_t*, hipStream_t);
template void launch_refresh_ap<float>(const Pools&, const int32_t*, int, int, int, int, double,
                                       int32_t*, hipStream_t);

}  // namespace mvmc
