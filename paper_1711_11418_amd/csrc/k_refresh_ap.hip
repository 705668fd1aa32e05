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

// Wider blocks (64 < n <= 16 NB): one workgroup of 16 x 16 threads per walker.
// Thread (ty, tx) keeps the tableau entries T[ty + 16 i][tx + 16 j],
// i, j < NB, in registers (a cyclic distribution, so every thread has work
// for any n).  Step k (column k): the threads of column k post the
// (threshold-)largest |T[r][k]| over their free rows as a 64-bit key through
// LDS; the pivot row p and column k go to LDS; every thread then applies the
// exchange step to its block:
//     T[p][k] <- 1/pi,   T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,   T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi.
// The column loop is split into an unrolled loop over the register column j
// and a runtime loop over the 16 thread columns, so every register index is
// a compile-time constant.
constexpr int kTileT = 16;            // thread grid side
constexpr int kTileThreads = kTileT * kTileT;

// Pivot key: the IEEE bits of |x| with the low seven mantissa bits replaced by
// 127 - row, so one unsigned maximum gives the largest magnitude (to 2^-45
// relative) and, among those, the lowest row; rows that may not be chosen
// have key 0.
__device__ __forceinline__ uint64_t tile_key(double x, int row, bool free_row) {
  const uint64_t b = (uint64_t)__double_as_longlong(fabs(x));
  return free_row ? ((b & ~(uint64_t)127) | (uint64_t)(127 - row)) : 0;
}

struct TileLds {
  double rowp[kTileT * 8];
  double colk[kTileT * 8];
  uint64_t keys[kTileT];
  double amax[kTileThreads / 64];
  int32_t piv[kTileT * 8];
  int32_t pinv[kTileT * 8];
};

template <typename T, int NB>
__global__ __launch_bounds__(kTileThreads, 2) void k_refresh_ap_tiled(
    Pools P, const int32_t* __restrict__ wlist, double sing_tol, int32_t* __restrict__ flags) {
  static_assert(NB <= 8, "tableau side at most 128");
  extern __shared__ __align__(16) unsigned char smem[];
  TileLds& L = *reinterpret_cast<TileLds*>(smem);
  int32_t* pos = reinterpret_cast<int32_t*>(smem + sizeof(TileLds));   // N_e
  const int gw = wlist[blockIdx.x];
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup;
  int32_t* occ = pos + ne;                                              // 2 N_s
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, tx = tid & (kTileT - 1), ty = tid / kTileT;

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = tid; b < ne; b += kTileThreads) pos[b] = posg[b];
  for (int v = tid; v < n2; v += kTileThreads) occ[v] = 0;
  __syncthreads();
  for (int b = tid; b < ne; b += kTileThreads) occ[pos[b]] = 1;

  // M[r][c] = f(site of up electron r, site of down electron c) = A[I_r][I_{n+c}]
  const double* A = P.A64 + I.A_off;
  double m[NB][NB];
  double amax = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int r = ty + kTileT * i;
    const int64_t roff = r < nh ? (int64_t)pos[r] * n2 : 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int c = tx + kTileT * j;
      const bool in = r < nh && c < nh;
      const double v = in ? A[roff + pos[nh + (in ? c : 0)]] : 0.0;
      m[i][j] = v;
      amax = fmax(amax, fabs(v));
    }
  }
  amax = wave_max(amax);
  if ((tid & 63) == 0) L.amax[tid / 64] = amax;
  __syncthreads();
  amax = fmax(fmax(L.amax[0], L.amax[1]), fmax(L.amax[2], L.amax[3]));
  const double tol = sing_tol * amax;

  uint32_t used = 0;   // bit i: row ty + 16 i already pivoted
  double mant = 1.0, minpiv = DBL_MAX, sgn = 1.0;
  int ex = 0;
  bool singular = false;
#pragma unroll
  for (int jk = 0; jk < NB; ++jk) {
    for (int txk = 0; txk < kTileT; ++txk) {
      const int k = kTileT * jk + txk;
      if (k >= nh || singular) break;   // uniform
      // pivot search over the free rows of column k
      if (tx == txk) {
        uint64_t key = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int r = ty + kTileT * i;
          const uint64_t kk = tile_key(m[i][jk], r, r < nh && !((used >> i) & 1u));
          key = kk > key ? kk : key;
        }
        L.keys[ty] = key;
#pragma unroll
        for (int i = 0; i < NB; ++i) L.colk[ty + kTileT * i] = m[i][jk];
      }
      __syncthreads();
      uint64_t kb = 0;
#pragma unroll
      for (int t = 0; t < kTileT; ++t) kb = L.keys[t] > kb ? L.keys[t] : kb;
      const double vmax = __longlong_as_double((long long)(kb & ~(uint64_t)127));
      if (kb == 0 || !(vmax > tol)) {
        singular = true;
        break;
      }
      const int p = 127 - (int)(kb & 127);
      const int pt = p & (kTileT - 1), pi = p / kTileT;
      if (ty == pt) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i == pi)
#pragma unroll
            for (int j = 0; j < NB; ++j) L.rowp[tx + kTileT * j] = m[i][j];
        used |= 1u << pi;
      }
      if (tid == 0) {
        L.piv[k] = p;
        L.pinv[p] = k;
      }
      __syncthreads();
      const double pv = L.colk[p];
      absdet_mul(mant, ex, fabs(pv));
      if (pv < 0.0) sgn = -sgn;
      minpiv = fmin(minpiv, fabs(pv));
      const double ip = 1.0 / pv;
      double rp[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) rp[j] = L.rowp[tx + kTileT * j];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int r = ty + kTileT * i;
        const bool isp = r == p;
        const double f = isp ? 0.0 : L.colk[r] * ip;
#pragma unroll
        for (int j = 0; j < NB; ++j) m[i][j] = isp ? -rp[j] * ip : fma(-f, rp[j], m[i][j]);
        if (tx == txk) m[i][jk] = isp ? ip : f;
      }
      __syncthreads();   // rowp, colk and keys are rewritten by the next step
    }
  }

  if (singular) {
    if (tid == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = -INFINITY;
      P.sgnpf[gw] = 0.0;
      P.minpiv[gw] = 0.0;
      P.status[gw] = 1;
    }
  } else {
    // sign of the pivot permutation k -> piv[k] (cycle lengths), then
    // Pf(X) = (-1)^{n(n-1)/2} det M
    if (tid == 0) {
      uint64_t seen[2] = {0, 0};
      int parity = 0;
      for (int b = 0; b < nh; ++b) {
        if ((seen[b >> 6] >> (b & 63)) & 1ull) continue;
        int c = b, len = 0;
        while (!((seen[c >> 6] >> (c & 63)) & 1ull)) {
          seen[c >> 6] |= 1ull << (c & 63);
          c = L.piv[c];
          ++len;
        }
        parity += len - 1;
      }
      if (parity & 1) sgn = -sgn;
      if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;
      if (flags) flags[gw] = 0;
      P.logpf[gw] = absdet_log(mant, ex);
      P.sgnpf[gw] = sgn;
      P.minpiv[gw] = minpiv / (amax > 0.0 ? amax : 1.0);
      P.status[gw] = 0;
    }
    // X^-1 = [[0, -M^-T], [M^-1, 0]] with M^-1[pinv[r]][piv[c]] = T[r][c]
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    for (int e = tid; e < ne * ne; e += kTileThreads) {
      const int r = e / ne, c = e - (e / ne) * ne;
      if ((r < nh) == (c < nh)) Y[e] = T(0);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int r = ty + kTileT * i;
      if (r >= nh) continue;
      const int a = L.pinv[r];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int c = tx + kTileT * j;
        if (c >= nh) continue;
        const int q = L.piv[c];
        Y[(int64_t)(nh + a) * ne + q] = (T)m[i][j];
        Y[(int64_t)q * ne + nh + a] = (T)(-m[i][j]);
      }
    }
  }

  // Jastrow field and RBM angles from scratch (v symmetric, W^T across threads)
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  for (int l = tid; l < ns; l += kTileThreads) {
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
    for (int hh = tid; hh < I.M; hh += kTileThreads) {
      double s = bb[hh];
      for (int v = 0; v < n2; ++v) s += WT[(int64_t)v * I.M + hh] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

__host__ __device__ inline size_t tiled_bytes(int max_ne, int max_sites) {
  return sizeof(TileLds) + (size_t)(max_ne + 2 * max_sites) * sizeof(int32_t);
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
    const size_t sh = (ap_walker_bytes(64, max_ns) + ap_minv_bytes<T>(wld)) * kApWpb;
    if (sh > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)&k_refresh_ap<T, 64>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh_ap<T, 64>), dim3(blocks), dim3(64 * kApWpb), sh, s, P, wlist, n,
                       max_ns, wld, sing_tol, flags);
  }
}

template void launch_refresh_ap<double>(const Pools&, const int32_t*, int, int, int, int, double,
                                        int32_t*, hipStream_t);
template void launch_refresh_ap<float>(const Pools&, const int32_t*, int, int, int, int, double,
                                       int32_t*, hipStream_t);

}  // namespace mvmc
