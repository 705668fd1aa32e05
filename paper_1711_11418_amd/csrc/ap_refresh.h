// Double-precision recomputation of a walker's state through the
// anti-parallel block of X (Eq. AP-Pf): device functions shared by the
// refresh kernels and the persistent sweep.
//
// With the n = N_e/2 up electrons first, X_ab = A[I_a][I_b] has zero
// same-spin blocks and the up-down block M[a][b] = f(site of up electron a,
// site of down electron b), so
//     X = [[0, M], [-M^T, 0]],   Pf(X) = (-1)^{n(n-1)/2} det M,
//     X^-1 = [[0, -M^-T], [M^-1, 0]].
// One wavefront per walker inverts M^T in place by Gauss-Jordan exchange
// steps with partial pivoting (det M^T = det M, (M^T)^-1 = (M^-1)^T; M^T
// loads one row of A per instruction).  Lane r keeps row r of the tableau T
// (= M^T at the start) in registers; the column loop is unrolled, so every
// register index is a compile-time constant.  Step k takes the unused row p of
// largest |T[r][k]|, pi = T[p][k], and exchanges row p with column k:
//     T[p][k] <- 1/pi,          T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,    T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi
// (r != p, c != k).  After all n steps T0^-1[a][p_b] = T[p_a][b] for the
// starting tableau T0 (here M^T, so M^-1[p_b][a] = T[p_a][b]), with p_k the
// pivot row of column k, and det M = det T0 = sgn(p) prod_k pi_k, the sign
// counted as the permutation is built.  The same pass recomputes the Jastrow field
// h_l = sum_m v_lm (n_m - 1) and the RBM angles theta = b + W sigma.
//
// ap_refresh_wave: one wavefront per walker (n <= NS <= 64).
// ap_refresh_tile: one workgroup of 16 x 16 threads per walker (n <= 16 NB),
// the exchange steps of ap_tile.h.
#pragma once

#include <float.h>

#include "ap_block.h"
#include "ap_tile.h"
#include "common.h"
#include "wave.h"

namespace mvmc {

namespace {
// dynamic LDS per walker: pos (2 NS ints), pivot row per column (NS ints),
// occupation (2 N_s ints)
__host__ __device__ inline size_t ap_walker_bytes(int ns_max, int nsmax_sites) {
  const size_t ints = (size_t)(2 * ns_max + ns_max + 2 * nsmax_sites);
  return (ints * sizeof(int32_t) + 15) & ~(size_t)15;
}

// LDS per walker for kMinvChunk rows of M^-1 at a time (row stride wld =
// max up electrons + 1), staged so X^-1 is written with the lanes across
// its rows.
constexpr int kMinvChunk = 16;
template <typename T>
__host__ __device__ inline size_t ap_minv_bytes(int wld) {
  return ((size_t)kMinvChunk * wld * sizeof(T) + 15) & ~(size_t)15;
}

// Walker gw by the calling wavefront (lane = threadIdx.x & 63); q: this
// wavefront's LDS (ap_walker_bytes(NS, max_sites) + ap_minv_bytes<T>(wld)).
// With flags, only when flags[gw] is set, which is then cleared.
template <typename T, int NS>
__device__ __forceinline__ void ap_refresh_wave(const Pools& P, int gw, unsigned char* q,
                                                int max_sites, int wld, double sing_tol,
                                                int32_t* __restrict__ flags) {
  using namespace wave;
  const int lane = threadIdx.x & 63;
  gw = sgpr(gw);
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup;
  const int64_t lw = gw - I.walker_off;

  int32_t* pos = (int32_t*)q;
  int32_t* piv = pos + 2 * NS;
  int32_t* occ = piv + NS;
  T* Wl = (T*)(q + ap_walker_bytes(NS, max_sites));   // M^-1, row stride wld

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = lane; b < ne; b += 64) pos[b] = posg[b];
  for (int v = lane; v < n2; v += 64) occ[v] = 0;
  wave_sync();
  for (int b = lane; b < ne; b += 64) occ[pos[b]] = 1;

  // The tableau is M^T: lane b keeps column b of M (the down electron b
  // against every up electron), so each load reads one row of A, the up
  // electron's, across the lanes.  det M^T = det M, and the elimination
  // yields (M^T)^-1 = (M^-1)^T.
  const double* A = P.A64 + I.A_off;
  const bool live = lane < nh;
  const int32_t col = live ? pos[nh + lane] : 0;
  double m[NS];
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    const bool in = live && c < nh;
    const double v = in ? A[(int64_t)pos[in ? c : 0] * n2 + col] : 0.0;
    m[c] = v;
    amax = fmax(amax, fabs(v));
  }
  amax = wave_max(amax);

  ApState st;
  ap_steps<0, NS>(st, m, piv, lane, live, nh, sing_tol * amax);
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
    // lane p_a holds row a of (M^T)^-1, i.e. column a of M^-1, at the
    // columns p_q.  Sixteen of them at a time, W[a - a0][q] = M^-1[q][a]
    // goes to LDS and the two non-zero blocks of Y are written with the
    // lanes across them:
    //   Y[a][n + q] = -W[a][q]  (rows of the upper-right block),
    //   Y[n + q][a] =  W[a][q]  (sixteen consecutive entries of each row n + q).
    // The same-spin blocks stay zero: the pool is cleared at init and no
    // kernel writes them.
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    int a = -1;   // row of the inverse pivoted by this lane's row
#pragma unroll
    for (int k = 0; k < NS; ++k)
      if (k < nh && piv[k] == lane) a = k;
    for (int a0 = 0; a0 < nh; a0 += kMinvChunk) {
      if (live && a >= a0 && a < a0 + kMinvChunk) {
#pragma unroll
        for (int b = 0; b < NS; ++b)
          if (b < nh) Wl[(a - a0) * wld + piv[b]] = (T)m[b];
      }
      wave_sync();
      const int na = nh - a0 < kMinvChunk ? nh - a0 : kMinvChunk;
      for (int rr = 0; rr < na; ++rr) {
        T* yr = Y + (int64_t)(a0 + rr) * ne + nh;
        for (int q = lane; q < nh; q += 64) yr[q] = -Wl[rr * wld + q];
      }
      for (int e = lane; e < nh * kMinvChunk; e += 64) {
        const int q = e / kMinvChunk, aa = e % kMinvChunk;
        if (aa < na) Y[(int64_t)(nh + q) * ne + a0 + aa] = Wl[aa * wld + q];
      }
      wave_sync();
    }
    if (lane == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = logabs;
      P.sgnpf[gw] = sgn;
      P.minpiv[gw] = minpiv / (amax > 0.0 ? amax : 1.0);
      P.status[gw] = 0;
    }
  }

  // Jastrow field (v symmetric: row m of V across the lanes is coalesced).
  // The sweeps keep it in double (exact adds of v differences), so a refresh
  // asked for by a flag (the periodic one, or after a non-finite ratio)
  // leaves it; the RBM angles, kept in the sweep precision, are redone.
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  if (!flags) {
    for (int l = lane; l < ns; l += 64) {
      double s = 0.0;
#pragma unroll 8
      for (int mm = 0; mm < ns; ++mm)
        s += V[(int64_t)mm * ns + l] * (double)(occ[mm] + occ[mm + ns] - 1);
      h[l] = s;
    }
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

// ---------------------------------------------------------------------------
// Two wavefronts per walker (32 < n <= 64): the tableau split by columns,
// wave w keeping the 32 columns [32 w, 32 w + 32) of every row (lane r, row
// r) in registers.  Step K: the wave holding column K picks the pivot row p
// (the same key and tie rule as ap_steps) and publishes p, pi and the
// multipliers f_r = T[r][K] / pi through LDS (double-buffered by the parity
// of K: one workgroup barrier per step); each wave then reads row p of its
// own columns from lane p (readlane) and updates them, and column K becomes
// f (row p: -1) with row p's scale -1/pi, as in ap_steps.
constexpr int kPairCols = 32;
constexpr int kPairThreads = 128;

struct PairLds {
  double f[2][64];
  double pv[2];
  double amax[2];
  int32_t p[2];
  int32_t piv[64];
};

// dynamic LDS of one walker: PairLds, pos (N_e), occupation (2 N_s) and
// M^-1 transposed (n x (n + 1) of T)
template <typename T>
__host__ __device__ inline size_t pair_bytes(int ne, int ns) {
  const int n = ne / 2;
  return ((sizeof(PairLds) + 15) & ~(size_t)15) +
         (((size_t)(ne + 2 * ns) * sizeof(int32_t) + 15) & ~(size_t)15) +
         (((size_t)n * (n + 1) * sizeof(T) + 15) & ~(size_t)15);
}

template <int K>
__device__ __forceinline__ void pair_steps(ApState& st, double (&m)[kPairCols], PairLds* L,
                                           int wid, int lane, bool live, int n, double tol,
                                           int& my_k) {
  if constexpr (K < 2 * kPairCols) {
    if (K >= n) return;
    constexpr int WK = K / kPairCols, CK = K % kPairCols;
    if (wid == WK) {
      const bool free_row = live && !((st.used >> lane) & 1ull);
      const uint32_t key = wave::wave_max_u32(wave::pivot_key32(m[CK], lane, free_row));
      const double vmax = wave::pivot_mag32(key);
      const int p = wave::pivot_lane32(key);
      const bool bad = key == 0 || !(vmax > tol) || p >= n;
      double pv = 0.0, f = 0.0;
      if (!bad) {
        const int xlo = __builtin_amdgcn_readlane(__double2loint(m[CK]), p);
        const int xhi = __builtin_amdgcn_readlane(__double2hiint(m[CK]), p);
        pv = __hiloint2double(xhi, xlo);
        f = lane == p ? 0.0 : m[CK] * (1.0 / pv);
      }
      L->f[K & 1][lane] = f;
      if (lane == 0) {
        L->p[K & 1] = bad ? -1 : p;
        L->pv[K & 1] = pv;
      }
    }
    __syncthreads();
    const int p = L->p[K & 1];
    if (p < 0) {
      st.singular = true;
      return;
    }
    const double pv = L->pv[K & 1];
    const double f = L->f[K & 1][lane];
    absdet_mul(st.mant, st.ex, fabs(pv));
    if (pv < 0.0) st.sgn = -st.sgn;
    st.minpiv = fmin(st.minpiv, fabs(pv));
    st.parity += __builtin_popcountll(~st.used & ((1ull << p) - 1ull));
    st.used |= 1ull << p;
    if (wid == 0 && lane == 0) L->piv[K] = p;
    const bool me = lane == p;
    if (me) my_k = K;
#pragma unroll
    for (int c = 0; c < kPairCols; ++c) {
      const int lo = __builtin_amdgcn_readlane(__double2loint(m[c]), p);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(m[c]), p);
      const double upd = fma(-f, __hiloint2double(hi, lo), m[c]);
      if (c == CK)
        m[c] = wid == WK ? (me ? -1.0 : f) : upd;
      else
        m[c] = upd;
    }
    if (me) st.rs = -1.0 / pv;
    pair_steps<K + 1>(st, m, L, wid, lane, live, n, tol, my_k);
  }
}

// Walker gw by a workgroup of kPairThreads threads (32 < n <= 64); smem:
// pair_bytes<T>(ne, ns).  With flags, only when flags[gw] is set, which is
// then cleared.  jastrow: recompute the Jastrow field too (the sweeps keep
// it in double, so the periodic refreshes skip it).  Contains workgroup
// barriers (uniform: one walker).
template <typename T>
__device__ __forceinline__ void ap_refresh_pair(const Pools& P, int gw, unsigned char* smem,
                                                double sing_tol, int32_t* __restrict__ flags,
                                                bool jastrow) {
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup, wld = nh + 1;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  PairLds* L = reinterpret_cast<PairLds*>(smem);
  int32_t* pos = reinterpret_cast<int32_t*>(smem + ((sizeof(PairLds) + 15) & ~(size_t)15));
  int32_t* occ = pos + ne;
  T* Wl = reinterpret_cast<T*>(
      smem + ((sizeof(PairLds) + 15) & ~(size_t)15) +
      ((((size_t)(ne + 2 * ns) * sizeof(int32_t)) + 15) & ~(size_t)15));   // Wl[a][q] = M^-1[q][a]

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = tid; b < ne; b += kPairThreads) pos[b] = posg[b];
  for (int v = tid; v < n2; v += kPairThreads) occ[v] = 0;
  __syncthreads();
  for (int b = tid; b < ne; b += kPairThreads) occ[pos[b]] = 1;

  // the tableau is M^T (lane b: down electron b against every up electron),
  // each load one row of A, the up electron's, across the lanes
  const double* A = P.A64 + I.A_off;
  const bool live = lane < nh;
  const int32_t col = live ? pos[nh + lane] : 0;
  double m[kPairCols];
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < kPairCols; ++c) {
    const int gc = wid * kPairCols + c;
    const bool in = live && gc < nh;
    const double v = in ? A[(int64_t)pos[in ? gc : 0] * n2 + col] : 0.0;
    m[c] = v;
    amax = fmax(amax, fabs(v));
  }
  amax = wave::wave_max(amax);
  if (lane == 0) L->amax[wid] = amax;
  __syncthreads();
  amax = fmax(L->amax[0], L->amax[1]);

  ApState st;
  int my_k = 0;
  pair_steps<0>(st, m, L, wid, lane, live, nh, sing_tol * amax, my_k);
  __syncthreads();   // piv[] for every thread
  if (st.singular) {
    if (tid == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = -INFINITY;
      P.sgnpf[gw] = 0.0;
      P.minpiv[gw] = 0.0;
      P.status[gw] = 1;
    }
  } else {
    const double logabs = absdet_log(st.mant, st.ex);
    double sgn = st.sgn;
    if (st.parity & 1) sgn = -sgn;
    if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;   // Pf(X) = (-1)^{n(n-1)/2} det M
    // lane r, pivot of step a = my_k, holds (M^T)^-1[a][p_b] = T[r][b], i.e.
    // M^-1[p_b][a]; through LDS the two non-zero blocks of Y are written
    // along their rows:  Y[a][n + q] = -M^-1[q][a],  Y[n + q][a] = M^-1[q][a].
    if (live) {
#pragma unroll
      for (int c = 0; c < kPairCols; ++c) {
        const int b = wid * kPairCols + c;
        if (b < nh) Wl[my_k * wld + L->piv[b]] = (T)(m[c] * st.rs);
      }
    }
    __syncthreads();
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    for (int e = tid; e < nh * nh; e += kPairThreads) {
      const int a = e / nh, q = e - a * nh;
      Y[(int64_t)a * ne + nh + q] = -Wl[a * wld + q];
    }
    for (int e = tid; e < nh * nh; e += kPairThreads) {
      const int q = e / nh, a = e - q * nh;
      Y[(int64_t)(nh + q) * ne + a] = Wl[a * wld + q];
    }
    if (tid == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = logabs;
      P.sgnpf[gw] = sgn;
      P.minpiv[gw] = st.minpiv / (amax > 0.0 ? amax : 1.0);
      P.status[gw] = 0;
    }
  }
  // Jastrow field (when asked) and RBM angles, as in ap_refresh_wave
  if (jastrow) {
    const double* V = P.V + I.V_off;
    double* h = P.h + I.h_off + lw * ns;
    for (int l = tid; l < ns; l += kPairThreads) {
      double s = 0.0;
#pragma unroll 8
      for (int mm = 0; mm < ns; ++mm)
        s += V[(int64_t)mm * ns + l] * (double)(occ[mm] + occ[mm + ns] - 1);
      h[l] = s;
    }
  }
  if (I.M) {
    const double* bb = P.rbm64 + I.rbm_b_off;
    const double* WT = P.rbmT64 + I.rbm_W_off;
    double* th = P.theta + I.theta_off + lw * I.M;
    for (int hh = tid; hh < I.M; hh += kPairThreads) {
      double s = bb[hh];
      for (int v = 0; v < n2; ++v) s += WT[(int64_t)v * I.M + hh] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

// Walker gw by the whole workgroup of kTileThreads threads (n <= 16 NB); smem:
// tiled_bytes(ne, ns).  With flags, only when flags[gw] is set, which is then
// cleared.  Contains workgroup barriers (uniform: the same gw everywhere).
template <typename T, int NB>
__device__ __forceinline__ void ap_refresh_tile(const Pools& P, int gw, unsigned char* smem,
                                                double sing_tol, int32_t* __restrict__ flags) {
  static_assert(NB <= 8, "tableau side at most 128");
  TileLds& L = *reinterpret_cast<TileLds*>(smem);
  int32_t* pos = reinterpret_cast<int32_t*>(smem + sizeof(TileLds));   // N_e
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

  double m[NB][NB];
  const double amax = tile_load<NB>(m, P.A64 + I.A_off, n2, pos, nh, tx, ty);
  const TileOut o = tile_invert<NB>(m, L, nh, amax, sing_tol);
  const bool singular = o.singular;

  if (singular) {
    if (tid == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = -INFINITY;
      P.sgnpf[gw] = 0.0;
      P.minpiv[gw] = 0.0;
      P.status[gw] = 1;
    }
  } else {
    if (tid == 0) {
      if (flags) flags[gw] = 0;
      P.logpf[gw] = o.logabs;
      P.sgnpf[gw] = tile_pf_sign(L, nh, o.sgn);
      P.minpiv[gw] = o.minpiv;
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

}  // namespace mvmc
