// Gauss-Jordan exchange steps on the anti-parallel block M of X, one
// wavefront per walker, lane r holding row r of the tableau (Eq. AP-Pf):
// with the up electrons first, X = [[0, M], [-M^T, 0]] with
// M[a][b] = f(site of up electron a, site of down electron b), so
// Pf(X) = (-1)^{n(n-1)/2} det M and X^-1 = [[0, -M^-T], [M^-1, 0]].
// Step k takes the unused row p of largest |T[r][k]| (to 2^-46 relative, the
// lowest such row), pi = T[p][k]:
//     T[p][k] <- 1/pi,          T[p][c] <- -T[p][c]/pi,
//     T[r][k] <- T[r][k]/pi,    T[r][c] <- T[r][c] - T[r][k] T[p][c]/pi,
// and after n steps M^-1[a][p_b] = T[p_a][b] (p_k the pivot row of column k),
// det M = sgn(p) prod_k pi_k.
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
  double mant = 1.0;   // |det| = mant 2^ex over the steps taken
  int ex = 0;
  uint64_t used = 0;   // rows pivoted so far
  int parity = 0;
  bool singular = false;
};

// Exchange step K (column K), then the next one: compile-time recursion, so
// every m[K] is a constant register index whatever the unroll heuristics.
// rowp: NS doubles of LDS for the pivot row; piv: NS ints, pivot row of each
// column.
template <int K, int NS>
__device__ __forceinline__ void ap_steps(ApState& st, double (&m)[NS], double* rowp,
                                         int32_t* piv, int lane, bool live, int nh,
                                         double tol) {
  if constexpr (K < NS) {
    if (K < nh && !st.singular) {
      const bool free_row = live && !((st.used >> lane) & 1ull);
      // one reduction for the largest |T[r][K]| over the free rows and its row
      const uint64_t key = wave::wave_max_u64(wave::pivot_key(m[K], lane, free_row));
      const double vmax = wave::pivot_mag(key);
      const int p = wave::pivot_lane(key);
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
        if (me)
#pragma unroll
          for (int c = 0; c < NS; ++c) rowp[c] = m[c];
        wave::wave_sync();
        const double ip = 1.0 / pv;
        const double t = m[K];
        const double g = me ? -ip : 1.0;
        const double f = me ? 0.0 : t * ip;
#pragma unroll
        for (int c = 0; c < NS; ++c)
          if (c != K) m[c] = fma(-f, rowp[c], g * m[c]);
        m[K] = me ? ip : t * ip;
        wave::wave_sync();
      }
    }
    ap_steps<K + 1, NS>(st, m, rowp, piv, lane, live, nh, tol);
  } else {
    st.logabs = absdet_log(st.mant, st.ex);
  }
}


}  // namespace
}  // namespace mvmc
