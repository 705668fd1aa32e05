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

// LDS-typed double, so that an address held in one VGPR (the asm barriers
// below) still addresses LDS with immediate offsets
typedef __attribute__((address_space(3))) double lds_double;

struct ApState {
  double logabs = 0.0, sgn = 1.0, minpiv = DBL_MAX;
  double rs = 1.0;     // this lane's deferred row scale s_r
  double mant = 1.0;   // |det| = mant 2^ex over the steps taken
  int ex = 0;
  uint64_t used = 0;   // rows pivoted so far
  int parity = 0;
  bool singular = false;
};

typedef __attribute__((address_space(3))) double lds_f64x2
    __attribute__((ext_vector_type(2)));

// Exchange step K (column K), then the next one: compile-time recursion, so
// every m[K] is a constant register index whatever the unroll heuristics.
// rowp: NS doubles of LDS for the pivot row (16-byte aligned); piv: NS ints,
// pivot row of each column.  CH: pivot-row values in flight per chunk
// (16-byte loads when even), bounded by the caller's register budget.
template <int K, int NS, int CH = (NS > 32 ? 4 : 8)>
__device__ __forceinline__ void ap_steps(ApState& st, double (&m)[NS], double* rowp,
                                         int32_t* piv, int lane, bool live, int nh,
                                         double tol) {
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
        if (me) {
          lds_double* wp = (lds_double*)rowp;
          asm volatile("" : "+v"(wp));
          if constexpr (NS % 2 == 0) {
            lds_f64x2* wp2 = (lds_f64x2*)wp;
#pragma unroll
            for (int c = 0; c < NS; c += 2) {
              lds_f64x2 v;
              v.x = m[c];
              v.y = m[c + 1];
              wp2[c / 2] = v;
            }
          } else {
#pragma unroll
            for (int c = 0; c < NS; ++c) wp[c] = m[c];
          }
        }
        // one wavefront's LDS operations complete in issue order, so the
        // reads below see the row without waiting for the writes: only the
        // compiler is kept from moving them
        asm volatile("" ::: "memory");
        const double ip = 1.0 / pv;
        const double f = me ? 0.0 : m[K] * ip;
        // the pivot row from one VGPR base with immediate offsets, CH values
        // in flight per chunk
        const lds_double* rp = (const lds_double*)rowp;
        asm volatile("" : "+v"(rp));
#pragma unroll
        for (int c0 = 0; c0 < NS; c0 += CH) {
          double r[CH];
          if constexpr (CH % 2 == 0 && NS % CH == 0) {
            const lds_f64x2* rp2 = (const lds_f64x2*)rp;
#pragma unroll
            for (int u = 0; u < CH; u += 2) {
              const lds_f64x2 v = rp2[(c0 + u) / 2];
              r[u] = v.x;
              r[u + 1] = v.y;
            }
          } else {
#pragma unroll
            for (int u = 0; u < CH; ++u) r[u] = c0 + u < NS ? rp[c0 + u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int c = c0 + u;
            if (c < NS && c != K) m[c] = fma(-f, r[u], m[c]);
          }
        }
        m[K] = me ? -1.0 : f;
        if (me) st.rs = -ip;
        asm volatile("" ::: "memory");   // next step's row write after these reads
      }
    }
    ap_steps<K + 1, NS, CH>(st, m, rowp, piv, lane, live, nh, tol);
  } else {
    st.logabs = absdet_log(st.mant, st.ex);
#pragma unroll
    for (int c = 0; c < NS; ++c) m[c] *= st.rs;   // T = s S
  }
}


}  // namespace
}  // namespace mvmc
