// Gauss-Jordan exchange steps on the anti-parallel block M of X, one
// wavefront per walker, lane r holding row r of the tableau (Eq. AP-Pf):
// with the up electrons first, X = [[0, M], [-M^T, 0]] with
// M[a][b] = f(site of up electron a, site of down electron b), so
// Pf(X) = (-1)^{n(n-1)/2} det M and X^-1 = [[0, -M^-T], [M^-1, 0]].
// Step k takes the unused row p of largest |T[r][k]| (to 2^-14 relative, the
// lowest such row: threshold partial pivoting), pi = T[p][k]:
//     T[p][k] <- 1/pi,          T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,    T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi,
// and after n steps M^-1[a][p_b] = T[p_a][b] (p_k the pivot row of column k),
// det M = sgn(p) prod_k pi_k.
// The pivot row's scaling by -1/pi is deferred: each lane keeps its row as
// T[r][.] = s_r S[r][.] with s_r = 1 until row r is chosen, then s_r = -1/pi
// and S[r][k] = -1 (its other entries unchanged).  A row that has not been
// chosen has T = S, so pi and the multipliers are read from S directly, and
// with f_r = S[r][k]/pi every other row takes
//     S[r][k] <- f_r,           S[r][c] <- S[r][c] - f_r S[p][c]
// (one fused multiply-add per entry); T = s S is formed after the last step.
#pragma once

#include <float.h>

#include "wave.h"

namespace mvmc {
namespace {

// |det M| is carried as a mantissa in [1/2, 1) and a binary exponent,
// renormalised after every pivot (one frexp per step instead of one
// logarithm); log|det M| is formed once, after the last step.
__device__ __forceinline__ void absdet_mul(double& mant, int& ex, double x) {
  int e;
  mant = frexp(mant * x, &e);
  ex += e;
}
__device__ __forceinline__ double absdet_log(double mant, int ex) {
  return log(mant) + (double)ex * 0.69314718055994530942;
}

struct ApState {
  double logabs = 0.0, sgn = 1.0, minpiv = DBL_MAX;
  double rs = 1.0;     // this lane's deferred row scale s_r
  double mant = 1.0;   // |det| = mant 2^ex over the steps taken
  int ex = 0;
  uint64_t used = 0;   // rows pivoted so far
  int parity = 0;
  bool singular = false;
};

// Exchange step K (column K), then the next one: compile-time recursion, so
// every m[K] is a constant register index whatever the unroll heuristics.
// piv: NS ints of LDS, pivot row of each column.
template <int K, int NS>
__device__ __forceinline__ void ap_steps(ApState& st, double (&m)[NS], int32_t* piv, int lane,
                                         bool live, int nh, double tol) {
  if constexpr (K < NS) {
    if (K < nh && !st.singular) {
      const bool free_row = live && !((st.used >> lane) & 1ull);
      // one reduction for the (threshold-)largest |T[r][K]| over the free rows
      // and its row
      const uint32_t key = wave::wave_max_u32(wave::pivot_key32(m[K], lane, free_row));
      const double vmax = wave::pivot_mag32(key);
      const int p = wave::pivot_lane32(key);
      if (key == 0 || !(vmax > tol) || p >= nh) {
        st.singular = true;
      } else {
        const int xlo = __builtin_amdgcn_readlane(__double2loint(m[K]), p);
        const int xhi = __builtin_amdgcn_readlane(__double2hiint(m[K]), p);
        const double pv = __hiloint2double(xhi, xlo);
        absdet_mul(st.mant, st.ex, fabs(pv));
        if (pv < 0.0) st.sgn = -st.sgn;
        st.minpiv = fmin(st.minpiv, fabs(pv));
        st.parity += __builtin_popcountll(~st.used & ((1ull << p) - 1ull));
        st.used |= 1ull << p;
        const bool me = lane == p;
        if (lane == 0) piv[K] = p;
        // the pivot row comes from lane p's registers as scalars (two
        // readlanes per entry, no LDS traffic: the LDS instruction queue is
        // what a wavefront waits on otherwise); lane p's own update is void
        // (f = 0), so reading entry c before its update is all that is needed
        const double ip = 1.0 / pv;
        const double f = me ? 0.0 : m[K] * ip;
#pragma unroll
        for (int c = 0; c < NS; ++c) {
          if (c == K) continue;
          const int lo = __builtin_amdgcn_readlane(__double2loint(m[c]), p);
          const int hi = __builtin_amdgcn_readlane(__double2hiint(m[c]), p);
          m[c] = fma(-f, __hiloint2double(hi, lo), m[c]);
        }
        m[K] = me ? -1.0 : f;
        if (me) st.rs = -ip;
      }
    }
    ap_steps<K + 1, NS>(st, m, piv, lane, live, nh, tol);
  } else {
    st.logabs = absdet_log(st.mant, st.ex);
#pragma unroll
    for (int c = 0; c < NS; ++c) m[c] *= st.rs;   // T = s S
  }
}


}  // namespace
}  // namespace mvmc
