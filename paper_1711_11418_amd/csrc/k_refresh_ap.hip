// Double-precision recomputation of a walker's state through the
// anti-parallel block of X (Eq. AP-Pf).
//
// With the n = N_e/2 up electrons first, X_ab = A[I_a][I_b] has zero
// same-spin blocks and the up-down block M[a][b] = f(site of up electron a,
// site of down electron b), so
//     X = [[0, M], [-M^T, 0]],   Pf(X) = (-1)^{n(n-1)/2} det M,
//     X^-1 = [[0, -M^-T], [M^-1, 0]].
// One wavefront per walker inverts M in place by Gauss-Jordan exchange
// steps with partial pivoting.  Lane r keeps row r of the tableau T (= M at
// the start) in registers; the column loop is unrolled, so every register
// index is a compile-time constant.  Step k takes the unused row p of
// largest |T[r][k]|, pi = T[p][k], and exchanges row p with column k:
//     T[p][k] <- 1/pi,          T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,    T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi
// (r != p, c != k).  After all n steps M^-1[a][p_b] = T[p_a][b], with p_k the
// pivot row of column k, and det M = sgn(p) prod_k pi_k, the sign counted as
// the permutation is built.  The same pass recomputes the Jastrow field
// h_l = sum_m v_lm (n_m - 1) and the RBM angles theta = b + W sigma.
#include <float.h>

#include "ap_block.h"
#include "launch.h"
#include "wave.h"

namespace mvmc {

namespace {
using namespace wave;
constexpr int kApWpb = 4;   // walkers (wavefronts) per workgroup

// dynamic LDS per walker: pos (2 NS ints), pivot row per column (NS ints),
// pivot row (NS doubles), occupation (2 N_s ints)
__host__ __device__ inline size_t ap_walker_bytes(int ns_max, int nsmax_sites) {
  const size_t ints = (size_t)(2 * ns_max + ns_max + 2 * nsmax_sites);
  return (ns_max * sizeof(double)) + ((ints * sizeof(int32_t) + 15) & ~(size_t)15);
}

// LDS per walker for M^-1 (row stride wld = max up electrons + 1), staged
// so X^-1 is written row by row with the lanes across the columns.
template <typename T>
__host__ __device__ inline size_t ap_minv_bytes(int wld) {
  return ((size_t)(wld - 1) * wld * sizeof(T) + 15) & ~(size_t)15;
}

template <typename T, int NS>
__global__ __launch_bounds__(64 * kApWpb, 2) void k_refresh_ap(Pools P,
                                                             const int32_t* __restrict__ wlist,
                                                             int n, int max_sites, int wld,
                                                             double sing_tol,
                                                             int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = blockIdx.x * kApWpb + wv;
  if (idx >= n) return;
  const int gw = sgpr(wlist[idx]);
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup;
  const int64_t lw = gw - I.walker_off;

  unsigned char* q = smem + (size_t)wv * (ap_walker_bytes(NS, max_sites) + ap_minv_bytes<T>(wld));
  double* rowp = (double*)q;
  int32_t* pos = (int32_t*)(rowp + NS);
  int32_t* piv = pos + 2 * NS;
  int32_t* occ = piv + NS;
  T* Wl = (T*)(q + ap_walker_bytes(NS, max_sites));   // M^-1, row stride wld

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = lane; b < ne; b += 64) pos[b] = posg[b];
  for (int v = lane; v < n2; v += 64) occ[v] = 0;
  wave_sync();
  for (int b = lane; b < ne; b += 64) occ[pos[b]] = 1;

  // row `lane` of M: the up electron `lane` against every down electron
  const double* A = P.A64 + I.A_off;
  const bool live = lane < nh;
  const int64_t roff = live ? (int64_t)pos[lane] * n2 : 0;
  double m[NS];
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    const bool in = live && c < nh;
    const double v = in ? A[roff + pos[nh + (in ? c : 0)]] : 0.0;
    m[c] = v;
    amax = fmax(amax, fabs(v));
  }
  amax = wave_max(amax);

  ApState st;
  ap_steps<0, NS>(st, m, rowp, piv, lane, live, nh, sing_tol * amax);
  double logabs = st.logabs, sgn = st.sgn, minpiv = st.minpiv;
  const int parity = st.parity;
  const bool singular = st.singular;

  if (singular) {
    if (lane == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = -INFINITY;
      P.sgnpf[gw] = 0.0;
      P.minpiv[gw] = 0.0;
      P.status[gw] = 1;
    }
  } else {
    if (parity & 1) sgn = -sgn;
    if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;   // Pf(X) = (-1)^{n(n-1)/2} det M
    // lane p_a holds row a of M^-1 at the columns p_b; W[a][q] = M^-1[a][q]
    // goes to LDS, then every row of Y is written with the lanes across it:
    //   Y[q][n + a] = -W[a][q],  Y[n + a][q] = W[a][q],  same-spin blocks 0
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    int a = -1;   // row of M^-1 pivoted by this lane's row
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (k < nh && piv[k] == lane) a = k;
    if (live && a >= 0) {
#pragma unroll
      for (int b = 0; b < NS; ++b)
        if (b < nh) Wl[a * wld + piv[b]] = (T)m[b];
    }
    wave_sync();
    for (int r = 0; r < ne; ++r) {
      T* yr = Y + (int64_t)r * ne;
      for (int c = lane; c < ne; c += 64) {
        T v = T(0);
        if (r < nh && c >= nh) v = -Wl[(c - nh) * wld + r];
        if (r >= nh && c < nh) v = Wl[(r - nh) * wld + c];
        yr[c] = v;
      }
    }
    if (lane == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = logabs;
      P.sgnpf[gw] = sgn;
      P.minpiv[gw] = minpiv / (amax > 0.0 ? amax : 1.0);
      P.status[gw] = 0;
    }
  }

  // Jastrow field (v symmetric: row m of V across the lanes is coalesced)
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  for (int l = lane; l < ns; l += 64) {
    double s = 0.0;
#pragma unroll 8
    for (int mm = 0; mm < ns; ++mm)
      s += V[(int64_t)mm * ns + l] * (double)(occ[mm] + occ[mm + ns] - 1);
    h[l] = s;
  }
  // RBM angles theta_h = b_h + sum_v W_hv (2 n_v - 1), W^T read across the lanes
  if (I.M) {
    const double* bb = P.rbm64 + I.rbm_b_off;
    const double* WT = P.rbmT64 + I.rbm_W_off;
    double* th = P.theta + I.theta_off + lw * I.M;
    for (int hh = lane; hh < I.M; hh += 64) {
      double s = bb[hh];
      for (int v = 0; v < n2; ++v) s += WT[(int64_t)v * I.M + hh] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

// Two or more wavefronts per walker (up to 64 NW rows of M, one per lane):
// the same exchange steps with the pivot search and the pivot row passed
// through LDS between workgroup barriers.
struct ApStateBlk {
  double logabs = 0.0, sgn = 1.0, minpiv = DBL_MAX;
  double mant = 1.0;   // |det| = mant 2^ex over the steps taken
  int ex = 0;
  uint64_t used[2] = {0, 0};   // rows pivoted so far (up to 128)
  int parity = 0;
  bool singular = false;
};

template <int K, int NS, int NW>
__device__ __forceinline__ void ap_steps_blk(ApStateBlk& st, double (&m)[NS], double* rowp,
                                             int32_t* piv, double* redv,
                                             int row, bool live, int nh, double tol) {
  if constexpr (K < NS) {
    if (K < nh && !st.singular) {
      const int lane = row & 63, wv = row >> 6;
      const bool free_row = live && !((st.used[row >> 6] >> (row & 63)) & 1ull);
      // per wavefront one reduction of the pivot key (largest |T[r][K]|, then
      // lowest row); the wavefronts' keys go through LDS as raw bits
      const uint64_t kw = wave_max_u64(pivot_key(m[K], lane, free_row));
      if (lane == 0) redv[wv] = __longlong_as_double((long long)kw);
      __syncthreads();
      uint64_t kbest = 0;
      int wbest = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t k = (uint64_t)__double_as_longlong(redv[w]);
        if (k > kbest) {
          kbest = k;
          wbest = w;
        }
      }
      const double vmax = pivot_mag(kbest);
      const int p = wbest * 64 + pivot_lane(kbest);
      if (kbest == 0 || !(vmax > tol) || p >= nh) {
        st.singular = true;
      } else {
        const bool me = row == p;
        if (me)
#pragma unroll
          for (int c = 0; c < NS; ++c) rowp[c] = m[c];
        if (threadIdx.x == 0) piv[K] = p;
        __syncthreads();
        const double pv = rowp[K];
        absdet_mul(st.mant, st.ex, fabs(pv));
        if (pv < 0.0) st.sgn = -st.sgn;
        st.minpiv = fmin(st.minpiv, fabs(pv));
        const int pl = p & 63, pwv = p >> 6;
        const uint64_t below = (1ull << pl) - 1ull;
        st.parity += __builtin_popcountll(~st.used[pwv] & below);
        if (pwv == 1) st.parity += __builtin_popcountll(~st.used[0]);
        st.used[pwv] |= 1ull << pl;
        const double ip = 1.0 / pv;
        const double t = m[K];
        const double g = me ? -ip : 1.0;
        const double f = me ? 0.0 : t * ip;
#pragma unroll
        for (int c = 0; c < NS; ++c)
          if (c != K) m[c] = fma(-f, rowp[c], g * m[c]);
        m[K] = me ? ip : t * ip;
        __syncthreads();   // rowp and the reduction slots are reused next step
      }
    }
    ap_steps_blk<K + 1, NS, NW>(st, m, rowp, piv, redv, row, live, nh, tol);
  } else {
    st.logabs = absdet_log(st.mant, st.ex);
  }
}

template <typename T, int NS, int NW>
__global__ __launch_bounds__(64 * NW) void k_refresh_ap_blk(Pools P,
                                                             const int32_t* __restrict__ wlist,
                                                             double sing_tol,
                                                             int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup;
  const int64_t lw = gw - I.walker_off;
  const int row = threadIdx.x, lane = row & 63;
  double* rowp = (double*)smem;                 // NS
  double* redv = rowp + NS;                     // NW
  int32_t* pos = (int32_t*)(redv + NW);         // 2 NS
  int32_t* piv = pos + 2 * NS;                  // NS
  int32_t* occ = piv + NS;                      // 2 N_s

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = row; b < ne; b += 64 * NW) pos[b] = posg[b];
  for (int v = row; v < n2; v += 64 * NW) occ[v] = 0;
  __syncthreads();
  for (int b = row; b < ne; b += 64 * NW) occ[pos[b]] = 1;

  const double* A = P.A64 + I.A_off;
  const bool live = row < nh;
  const int64_t roff = live ? (int64_t)pos[row] * n2 : 0;
  double m[NS];
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    const bool in = live && c < nh;
    const double v = in ? A[roff + pos[nh + (in ? c : 0)]] : 0.0;
    m[c] = v;
    amax = fmax(amax, fabs(v));
  }
  amax = wave_max(amax);
  if (lane == 0) redv[row >> 6] = amax;
  __syncthreads();
  amax = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) amax = fmax(amax, redv[w]);
  __syncthreads();

  ApStateBlk st;
  ap_steps_blk<0, NS, NW>(st, m, rowp, piv, redv, row, live, nh, sing_tol * amax);
  __syncthreads();
  if (st.singular) {
    if (row == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = -INFINITY;
      P.sgnpf[gw] = 0.0;
      P.minpiv[gw] = 0.0;
      P.status[gw] = 1;
    }
  } else {
    double sgn = st.sgn;
    if (st.parity & 1) sgn = -sgn;
    if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    int a = -1;
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (k < nh && piv[k] == row) a = k;
    if (live && a >= 0) {
      T* rdn = Y + (int64_t)(nh + a) * ne;
      for (int b = 0; b < nh; ++b) rdn[nh + b] = T(0);
#pragma unroll
      for (int b = 0; b < NS; ++b)
        if (b < nh) {
          const int qb = piv[b];
          rdn[qb] = (T)m[b];
          Y[(int64_t)qb * ne + nh + a] = (T)(-m[b]);
        }
    }
    if (live) {
      T* rup = Y + (int64_t)row * ne;
      for (int b = 0; b < nh; ++b) rup[b] = T(0);
    }
    if (row == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = st.logabs;
      P.sgnpf[gw] = sgn;
      P.minpiv[gw] = st.minpiv / (amax > 0.0 ? amax : 1.0);
      P.status[gw] = 0;
    }
  }
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  for (int l = row; l < ns; l += 64 * NW) {
    double s = 0.0;
#pragma unroll 8
    for (int mm = 0; mm < ns; ++mm)
      s += V[(int64_t)mm * ns + l] * (double)(occ[mm] + occ[mm + ns] - 1);
    h[l] = s;
  }
  if (I.M) {
    const double* bb = P.rbm64 + I.rbm_b_off;
    const double* WT = P.rbmT64 + I.rbm_W_off;
    double* th = P.theta + I.theta_off + lw * I.M;
    for (int hh = row; hh < I.M; hh += 64 * NW) {
      double s = bb[hh];
      for (int v = 0; v < n2; ++v) s += WT[(int64_t)v * I.M + hh] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

__host__ __device__ inline size_t ap_blk_bytes(int NS, int NW, int max_sites) {
  return (size_t)(NS + NW) * sizeof(double) +
         (size_t)(2 * NS + NS + 2 * max_sites) * sizeof(int32_t);
}
}  // namespace

bool refresh_ap_fits(int max_ne, int max_ns) {
  if (max_ne <= 128)
    return (ap_walker_bytes(64, max_ns) + ap_minv_bytes<double>(max_ne / 2 + 1)) * kApWpb <=
           152 * 1024;
  return max_ne <= 160 && ap_blk_bytes(80, 2, max_ns) <= 64 * 1024;
}

template <typename T>
void launch_refresh_ap(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                       double sing_tol, int32_t* flags, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (n + kApWpb - 1) / kApWpb;
  if (max_ne > 128) {   // up to 80 electrons per spin: two wavefronts per walker
    const size_t sh = ap_blk_bytes(80, 2, max_ns);
    hipLaunchKernelGGL((k_refresh_ap_blk<T, 80, 2>), dim3(n), dim3(128), sh, s, P, wlist,
                       sing_tol, flags);
    return;
  }
  const int wld = max_ne / 2 + 1;
  if (max_ne <= 64) {
    const size_t sh = (ap_walker_bytes(32, max_ns) + ap_minv_bytes<T>(wld)) * kApWpb;
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)&k_refresh_ap<T, 32>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh_ap<T, 32>), dim3(blocks), dim3(64 * kApWpb), sh, s, P, wlist, n,
                       max_ns, wld, sing_tol, flags);
  } else {
    const size_t sh = (ap_walker_bytes(64, max_ns) + ap_minv_bytes<T>(wld)) * kApWpb;
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)&k_refresh_ap<T, 64>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh_ap<T, 64>), dim3(blocks), dim3(64 * kApWpb), sh, s, P, wlist, n,
                       max_ns, wld, sing_tol, flags);
  }
}

template void launch_refresh_ap<double>(const Pools&, const int32_t*, int, int, int, double,
                                        int32_t*, hipStream_t);
template void launch_refresh_ap<float>(const Pools&, const int32_t*, int, int, int, double,
                                       int32_t*, hipStream_t);

}  // namespace mvmc
