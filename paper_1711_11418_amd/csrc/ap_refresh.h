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
// pivot row (NS doubles), occupation (2 N_s ints)
__host__ __device__ inline size_t ap_walker_bytes(int ns_max, int nsmax_sites) {
  const size_t ints = (size_t)(2 * ns_max + ns_max + 2 * nsmax_sites);
  return (ns_max * sizeof(double)) + ((ints * sizeof(int32_t) + 15) & ~(size_t)15);
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
  ap_steps<0, NS, (NS > 32 ? 32 : NS)>(st, m, rowp, piv, lane, live, nh, sing_tol * amax);
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
