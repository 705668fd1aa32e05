// Gauss-Jordan exchange steps on the anti-parallel block M of X (Eq. AP-Pf)
// by one workgroup of 16 x 16 threads per walker, for 64 < n <= 16 NB, and
// inside the anti-parallel-block sweep for any n <= 16 NB.
//
// With the up electrons first, X = [[0, M], [-M^T, 0]] with
// M[a][b] = f(site of up electron a, site of down electron b), so
// Pf(X) = (-1)^{n(n-1)/2} det M and X^-1 = [[0, -M^-T], [M^-1, 0]].
// Thread (ty, tx) keeps the tableau entries T[ty + 16 i][tx + 16 j],
// i, j < NB, in registers (a cyclic distribution, so every thread has work
// for any n).  Step k (column k): the threads of column k post the
// (threshold-)largest |T[r][k]| over their free rows as a 64-bit key through
// LDS; the pivot row p and column k go to LDS; every thread then applies the
// exchange step to its block:
//     T[p][k] <- 1/pi,   T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,   T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi.
// After n steps M^-1[pinv[r]][piv[c]] = T[r][c] (piv[k] the pivot row of
// column k, pinv its inverse) and det M = sgn(piv) prod_k pi_k.  The column
// loop is split into an unrolled loop over the register column j and a
// runtime loop over the 16 thread columns, so every register index is a
// compile-time constant.  The arithmetic of an entry does not depend on NB.
#pragma once

#include <float.h>

#include "ap_block.h"
#include "common.h"
#include "wave.h"

namespace mvmc {
namespace {

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

struct TileOut {
  bool singular;
  double logabs;   // log |det M|
  double sgn;      // sign of the product of the pivots (the permutation not yet counted)
  double minpiv;   // smallest |pivot| / max |M|
};

// m[i][j] = M[ty + 16 i][tx + 16 j] (0 outside n x n) from the spin-orbitals
// pos[0, 2n) (up electrons first) and the double table A (row stride n2);
// returns this thread's largest |entry|.
template <int NB>
__device__ __forceinline__ double tile_load(double (&m)[NB][NB], const double* __restrict__ A,
                                            int n2, const int32_t* pos, int nh, int tx, int ty) {
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
  return amax;
}

// The n exchange steps.  Every thread of the workgroup calls it with the
// same nh; contains workgroup barriers; the result is the same in every
// thread, and L.piv / L.pinv hold the pivot rows when it returns.
template <int NB>
__device__ __forceinline__ TileOut tile_invert(double (&m)[NB][NB], TileLds& L, int nh,
                                               double amax, double sing_tol) {
  const int tid = threadIdx.x, tx = tid & (kTileT - 1), ty = tid / kTileT;
  amax = wave::wave_max(amax);
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
  TileOut o;
  o.singular = singular;
  o.logabs = singular ? -INFINITY : absdet_log(mant, ex);
  o.sgn = sgn;
  o.minpiv = singular ? 0.0 : minpiv / (amax > 0.0 ? amax : 1.0);
  return o;
}

// Sign of Pf(X) from the sign of the pivot product: the parity of the pivot
// permutation k -> piv[k] (cycle lengths), then Pf(X) = (-1)^{n(n-1)/2} det M.
// One thread.
__device__ __forceinline__ double tile_pf_sign(const TileLds& L, int nh, double sgn) {
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
  return sgn;
}

}  // namespace
}  // namespace mvmc
