// Metropolis proposals of one walker on the anti-parallel block alone: one
// workgroup keeps only M^-1 (n x n, n = N_e/2) in LDS for the whole run.
//
// With the up electrons first and the anti-parallel pair amplitude
// (Eq. AP-Pf), X = [[0, M], [-M^T, 0]] with M[i][b] = f(site of up electron i,
// site of down electron b), Pf(X) = (-1)^{n(n-1)/2} det M and
// X^-1 = [[0, -M^-T], [M^-1, 0]]: the other three blocks of X^-1 are zero or
// carry the same numbers, so M^-1 is the whole state.  The hopping update of
// section 3.1.2 then changes one row or one column of M, and the Pfaffian
// ratio and the new inverse follow from the matrix-determinant lemma and
// Sherman-Morrison (the fast update the paper defers to its references):
//
//   up electron a moves to site s':   m'[b] = f(s', s_b) (new row a of M)
//     r = sum_b m'[b] M^-1[b][a],   v[j] = sum_b m'[b] M^-1[b][j] - delta_ja,
//     M^-1 <- M^-1 - M^-1[:, a] v^T / r
//   down electron b0 moves to s':     m'[i] = f(s_i, s') (new column b0 of M)
//     r = sum_i M^-1[b0][i] m'[i],  t[i] = sum_j M^-1[i][j] m'[j] - delta_i,b0,
//     M^-1 <- M^-1 - t M^-1[b0, :] / r
//
// A proposal reads one column or row of M^-1 (n w bytes); an accepted one
// reads M^-1 once for v or t and reads and writes it once for the rank-1
// update (3 n^2 w bytes).  The walker's M^-1 is read from the lower-left
// block of its X^-1 and both non-zero blocks are written back at the end, so
// every other kernel sees the usual X^-1.
//
// Exchange update (section 3.1.2, Fig. 5b): up electron a (site i) and down
// electron b (site j) trade sites, so row a and column b of M change at once:
// M' = M + e_a u^T + w e_b^T with u the change of row a (its entry b included)
// and w the change of column b off row a.  With
//   rho   = sum_b' r'[b'] M^-1[b'][a]    r' the new row a (r'[b] = f(j, i))
//   sigma = sum_a' M^-1[b][a'] c[a']     c the new column b off row a, c[a] = f(i, j)
//   t'    = M^-1 c,   beta = u . t' - u[b],   gamma = M^-1[b][a]
// the determinant lemma gives det M'/det M = rho sigma - beta gamma, and the
// Woodbury identity the rank-2 update
//   M^-1 <- M^-1 - M^-1[:, a] l1^T - (t' - e_b) l2^T,
//   l1 = (sigma s - beta M^-1[b, :]) / D,  l2 = (rho M^-1[b, :] - gamma s) / D,
// s = u^T M^-1, D the ratio.  Charges per site do not change, so the
// Gutzwiller and Jastrow factors stay; four RBM visibles flip.
//
// The walker stops at every multiple of refresh_every (of its proposal
// counter, or of its applied-update counter when the pools say so) and at a
// non-finite ratio (guard word kGuardPending; a second one in a row, after
// the double-precision refresh, gives kGuardFailed) and reports whether it
// stopped for a refresh.
#pragma once

#include "common.h"

namespace mvmc {

namespace {
struct ApSweepLds {
  size_t Mi, vec, part, h, th, red, ints, total;
  int ld;
};
__host__ __device__ inline size_t ap16(size_t x) { return (x + 15) & ~(size_t)15; }
// Row stride n + 1 (odd for even n): the strided column reads of the ratio of
// an up move and of t for a down move spread over the LDS banks.
__host__ __device__ inline ApSweepLds ap_sweep_layout(int ne, int ns, int M, size_t ts, int nw) {
  ApSweepLds L;
  const int n = ne / 2;
  L.ld = n + ((n & 1) ? 0 : 1);
  L.Mi = ap16((size_t)n * L.ld * ts);
  L.vec = ap16(8 * (size_t)n * ts);             // hop: m', column/row, v or t; exchange: 8
  L.part = ap16((size_t)nw * n * ts);           // partial sums of v or t per wavefront
  L.h = ap16((size_t)ns * sizeof(double));
  L.th = ap16((size_t)M * ts);
  L.red = ap16(2 * (size_t)(nw > 8 ? nw : 8) * sizeof(double));
  L.ints = ap16((size_t)(ne + 4 * ns + 2) * sizeof(int32_t));
  L.total = L.Mi + L.vec + L.part + L.h + L.th + L.red + L.ints;
  return L;
}

template <typename T> __device__ __forceinline__ const T* ap_table(const Pools& P, int64_t off);
template <> __device__ __forceinline__ const double* ap_table<double>(const Pools& P, int64_t off) {
  return P.A64 + off;
}
template <> __device__ __forceinline__ const float* ap_table<float>(const Pools& P, int64_t off) {
  return P.A32 + off;
}
template <typename T> __device__ __forceinline__ const T* ap_rbm(const Pools& P);
template <> __device__ __forceinline__ const double* ap_rbm<double>(const Pools& P) { return P.rbm64; }
template <> __device__ __forceinline__ const float* ap_rbm<float>(const Pools& P) { return P.rbm32; }

// out = M^-1 x (rows) or out = x^T M^-1 (columns) over the n x n block: each
// wavefront sums a slice of the contraction index for every output index,
// the slices are then added in order.  Contains two workgroup barriers.
template <typename T, int NW, int NT>
__device__ __forceinline__ void ap_matvec(const T* Mi, int ld, int n, const T* x, T* out, T* part,
                                          bool rows) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int j0 = (wid * n) / NW, j1 = ((wid + 1) * n) / NW;
  for (int o = lane; o < n; o += 64) {
    T s = T(0);
    if (rows)
      for (int j = j0; j < j1; ++j) s += Mi[o * ld + j] * x[j];
    else
      for (int j = j0; j < j1; ++j) s += x[j] * Mi[j * ld + o];
    part[wid * n + o] = s;
  }
  __syncthreads();
  for (int o = tid; o < n; o += NT) {
    T s = T(0);
#pragma unroll
    for (int w = 0; w < NW; ++w) s += part[w * n + o];
    out[o] = s;
  }
  __syncthreads();
}

// The proposals of global walker gw up to target[gw], at most cap of them
// and only up to the next multiple of R (proposals, or applied updates).  Every thread of the workgroup calls
// it with the same gw; it contains workgroup barriers and returns the same
// value in every thread: true when the walker stopped for a refresh (at a
// multiple of R or at a non-finite ratio), when needs_refresh[gw] (if given)
// is also set.  smem: ap_sweep_layout.  FULL = false: no trace, no exchange
// updates and no RBM factor (the caller guarantees it), which leaves their
// code and its scalar state out of the loop.
template <typename T, int NT, bool FULL = true>
__device__ __forceinline__ bool ap_walk(const Pools& P, int gw, unsigned char* smem, int cap,
                                        uint64_t seed, TraceRec* trace, int64_t trace_cap,
                                        const uint64_t* __restrict__ trace_base,
                                        const uint64_t* __restrict__ target,
                                        int32_t* __restrict__ needs_refresh, int R, int ex64) {
  constexpr int NW = NT / 64;
  if constexpr (!FULL) {
    trace = nullptr;
    ex64 = 0;
  }
  const int32_t guard0 = P.guard[gw];
  if (guard0 == kGuardFailed) return false;
  const uint64_t n0 = P.cnt[gw];
  const uint64_t tg = target[gw];
  uint64_t todo = tg > n0 ? tg - n0 : 0;
  if (todo > (uint64_t)cap) todo = (uint64_t)cap;
  const bool by_upd = P.refresh_upd != 0;
  if (R > 0 && !by_upd) {
    const uint64_t left = (uint64_t)R - n0 % (uint64_t)R;
    if (todo > left) todo = left;
  }
  if (todo == 0) return false;
  const int n_prop = (int)todo;
  const uint64_t u0 = P.upd[gw];
  bool due = false;   // the applied update that completes a multiple of R was made
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, M = FULL ? I.M : 0, n = I.nup;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  const ApSweepLds L = ap_sweep_layout(ne, ns, M, sizeof(T), NW);
  const int ld = L.ld;
  unsigned char* q = smem;
  T* Mi = (T*)q;                 // M^-1[i][j] at i*ld + j
  q += L.Mi;
  T* mv = (T*)q;                 // m': new row (up move) or column (down move) of M
  T* cr = mv + n;                // column a (up) or row b0 (down) of M^-1
  T* vt = cr + n;                // v (up) or t (down)
  q += L.vec;
  T* part = (T*)q;               // [NW][n] partial sums of v or t
  q += L.part;
  double* hs = (double*)q;
  q += L.h;
  T* ths = (T*)q;
  q += L.th;
  double* red = (double*)q;
  q += L.red;
  int32_t* pos_s = (int32_t*)q;
  int32_t* eidx = pos_s + ne;    // 2ns: electron at spin-orbital, -1 empty
  int32_t* emp = eidx + n2;      // 2ns: empty lists [sigma][ns]
  int32_t* slot = emp + n2;      // 2: list slots of an exchange

  T* Yg = (T*)P.Y + I.Y_off + lw * ne * ne;
  int32_t* posg = P.pos + I.pos_off + lw * ne;
  int32_t* empg = P.empty + I.empty_off + lw * n2;
  double* hg = P.h + I.h_off + lw * ns;
  double* thg = P.theta + I.theta_off + lw * M;

  // M^-1[i][j] = X^-1[n + i][j]
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    Mi[i * ld + j] = Yg[(int64_t)(n + i) * ne + j];
  }
  for (int v = tid; v < n2; v += NT) {
    eidx[v] = -1;
    emp[v] = empg[v];
  }
  for (int l = tid; l < ns; l += NT) hs[l] = hg[l];
  for (int hh = tid; hh < M; hh += NT) ths[hh] = (T)thg[hh];
  __syncthreads();
  for (int b = tid; b < ne; b += NT) {
    const int v = posg[b];
    pos_s[b] = v;
    eidx[v] = b;
  }
  __syncthreads();

  const T* A = ap_table<T>(P, I.A_off);
  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const T* ra = ap_rbm<T>(P) + I.rbm_a_off;
  const T* rW = ap_rbm<T>(P) + I.rbm_W_off;
  const uint64_t tb = trace ? trace_base[gw] : 0;
  int64_t acc = 0;
  int32_t guard1 = guard0;

  int it = 0;
  // each proposal's draw is formed during the previous one (scalar work that
  // overlaps the previous proposal's loads)
  uint4 r_cur = draw(seed, n0, (uint32_t)gw, 0u);
  while (it < n_prop) {
    const uint64_t nn = n0 + (uint64_t)it;
    const uint4 r = r_cur;
    r_cur = draw(seed, nn + 1, (uint32_t)gw, 0u);
    bool nonfinite = false;
    do {   // one proposal; `continue` ends it
    if (ex64 && (int)(r.w & 63u) < ex64) {
      // ------------------------------------------------------ exchange
      const int a = scaled(r.x, n), bd = scaled(r.y, ne - n), b = n + bd;
      const int si = pos_s[a], sj = pos_s[b] - ns;
      if (si == sj || eidx[sj] >= 0 || eidx[si + ns] >= 0) {   // no such move
        if (trace && tid == 0 && nn - tb < (uint64_t)trace_cap) {
          TraceRec rec;
          rec.n = (int64_t)nn; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
          rec.ratio = 0.0; rec.b = b; rec.pad = 0;
          trace[(int64_t)gw * trace_cap + (int64_t)(nn - tb)] = rec;
        }
        continue;
      }
      T* rn = mv;            // new row a of M
      T* cn = mv + n;        // new column b off row a (c[a] = old M[a][b])
      T* uu = mv + 2 * n;    // change of row a
      T* ca = mv + 3 * n;    // column a of M^-1
      T* rb = mv + 4 * n;    // row b of M^-1
      T* tp = mv + 5 * n;    // t' = M^-1 c
      T* l1 = mv + 6 * n;
      T* l2 = mv + 7 * n;
      const T* Ai = A + (int64_t)si * n2 + ns;   // f(i, .)
      const T* Aj = A + (int64_t)sj * n2 + ns;   // f(j, .)
      T accr = T(0), accs = T(0);
      for (int q2 = tid; q2 < n; q2 += NT) {
        const int sb = pos_s[n + q2] - ns;
        const T fn = q2 == bd ? Aj[si] : Aj[sb];
        const T c = Mi[q2 * ld + a];
        rn[q2] = fn;
        uu[q2] = fn - Ai[sb];
        ca[q2] = c;
        accr += fn * c;
        const int s_up = pos_s[q2];
        const T cv = q2 == a ? Ai[sj] : -A[(int64_t)(ns + si) * n2 + s_up];   // f(s_up, i), row-wise
        const T rv = Mi[bd * ld + q2];
        cn[q2] = cv;
        rb[q2] = rv;
        accs += rv * cv;
      }
      double accm = 0.0;
      if (M) {
        for (int hh = tid; hh < M; hh += NT) {
          const T* Wh = rW + (int64_t)hh * n2;
          const T d = T(2) * (Wh[sj] - Wh[si] + Wh[si + ns] - Wh[sj + ns]);
          const T th = ths[hh];
          accm += (double)(log2cosh(th + d) - log2cosh(th));
        }
      }
      double rho = (double)accr, sig = (double)accs;
      block_sum2(rho, sig, red);
      accm = block_sum(accm, red);
      __syncthreads();   // the vectors above, for every thread
      const double gam = (double)Mi[bd * ld + a];
      ap_matvec<T, NW, NT>(Mi, ld, n, cn, tp, part, true);
      T accb = T(0);
      for (int q2 = tid; q2 < n; q2 += NT) accb += uu[q2] * tp[q2];
      double bet = (double)accb;
      bet = block_sum(bet, red) - (double)uu[bd];
      const double D = rho * sig - bet * gam;
      double logc = 0.0;
      if (M) logc = 2.0 * ((double)ra[sj] - (double)ra[si] + (double)ra[si + ns] -
                           (double)ra[sj + ns]) + accm;
      const double Rt = D * exp(logc);
      if (!isfinite(Rt)) {   // uniform: every thread holds the same sums
        nonfinite = true;
        continue;
      }
      guard1 = kGuardClear;
      const bool accept = uniform53(r.z, r.w) < Rt * Rt;
      if (trace && tid == 0 && nn - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.n = (int64_t)nn; rec.walker = gw; rec.a = a; rec.i_new = sj;
        rec.accepted = accept ? 1 : 0; rec.ratio = Rt; rec.b = b; rec.pad = 0;
        trace[(int64_t)gw * trace_cap + (int64_t)(nn - tb)] = rec;
      }
      if (!accept) continue;
      ++acc;
      due = by_upd && R > 0 && (u0 + (uint64_t)acc) % (uint64_t)R == 0;
      ap_matvec<T, NW, NT>(Mi, ld, n, uu, l1, part, false);   // s = u^T M^-1 (into l1)
      const double iD = 1.0 / D;
      for (int q2 = tid; q2 < n; q2 += NT) {
        const double sv = (double)l1[q2], rv = (double)rb[q2];
        l2[q2] = (T)((rho * rv - gam * sv) * iD);
        l1[q2] = (T)((sig * sv - bet * rv) * iD);
      }
      // list slots of j (up list) and i (down list)
      for (int q2 = tid; q2 < ns; q2 += NT) {
        if (emp[q2] == sj) slot[0] = q2;
        if (emp[ns + q2] == si) slot[1] = q2;
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += NT) {
        const int i2 = e / n, j2 = e - (e / n) * n;
        const T tv = tp[i2] - (i2 == bd ? T(1) : T(0));
        Mi[i2 * ld + j2] -= ca[i2] * l1[j2] + tv * l2[j2];
      }
      for (int hh = tid; hh < M; hh += NT) {
        const T* Wh = rW + (int64_t)hh * n2;
        ths[hh] += T(2) * (Wh[sj] - Wh[si] + Wh[si + ns] - Wh[sj + ns]);
      }
      if (tid == 0) {
        pos_s[a] = sj;
        pos_s[b] = si + ns;
        eidx[si] = -1;
        eidx[sj + ns] = -1;
        eidx[sj] = a;
        eidx[si + ns] = b;
        emp[slot[0]] = si;
        emp[ns + slot[1]] = sj;
      }
      __syncthreads();
      continue;
    }
    const int a = scaled(r.x, ne);
    const int sigma = a >= n ? 1 : 0;
    const int nemp = ns - (sigma ? I.ndn : n);
    if (nemp == 0) {
      if (trace && tid == 0 && nn - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.b = -1; rec.pad = 0;
        rec.n = (int64_t)nn; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
        rec.ratio = 0.0;
        trace[(int64_t)gw * trace_cap + (int64_t)(nn - tb)] = rec;
      }
      continue;
    }
    const int k = scaled(r.y, nemp);
    const int site_new = emp[sigma * ns + k];
    const int Inew = site_new + sigma * ns;
    const int Iold = pos_s[a];
    const int site_old = Iold - sigma * ns;
    const int ai = a - sigma * n;   // row of M (up) or column of M (down)

    // m' and the ratio; the column (up) or row (down) of M^-1 it reads is
    // kept for the update
    T accp = T(0);
    if (sigma == 0) {
      const T* Arow = A + (int64_t)Inew * n2;   // f(s', s_b) = A[(s', up)][(s_b, dn)]
      for (int b = tid; b < n; b += NT) {
        const T x = Arow[pos_s[n + b]];
        const T c = Mi[b * ld + ai];
        mv[b] = x;
        cr[b] = c;
        accp += x * c;
      }
    } else {
      for (int i = tid; i < n; i += NT) {
        // f(s_i, s') = A[(s_i, up)][(s', dn)] = -A[(s', dn)][(s_i, up)]: one row of
        // the skew table across the threads instead of a column
        const T x = -A[(int64_t)Inew * n2 + pos_s[i]];
        const T c = Mi[ai * ld + i];
        mv[i] = x;
        cr[i] = c;
        accp += c * x;
      }
    }
    double accr = 0.0;
    if (M) {
      for (int hh = tid; hh < M; hh += NT) {
        const T d = T(2) * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
        const T th = ths[hh];
        accr += (double)(log2cosh(th + d) - log2cosh(th));
      }
    }
    double sp = (double)accp, sr = accr;
    block_sum2(sp, sr, red);
    const double r_pf = sp;
    const int opp = (1 - sigma) * ns;
    double logc = G[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  G[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                  hs[site_old] - V[(int64_t)site_old * ns + site_new];
    if (M) logc += 2.0 * ((double)ra[Inew] - (double)ra[Iold]) + sr;
    const double Rt = r_pf * exp(logc);
    if (!isfinite(Rt)) {   // uniform: every thread holds the same sums
      nonfinite = true;
      continue;
    }
    guard1 = kGuardClear;
    const double u = uniform53(r.z, r.w);
    const bool accept = u < Rt * Rt;
    if (trace && tid == 0 && nn - tb < (uint64_t)trace_cap) {
      TraceRec rec;
      rec.b = -1; rec.pad = 0;
      rec.n = (int64_t)nn; rec.walker = gw; rec.a = a; rec.i_new = Inew;
      rec.accepted = accept ? 1 : 0; rec.ratio = Rt;
      trace[(int64_t)gw * trace_cap + (int64_t)(nn - tb)] = rec;
    }
    if (!accept) continue;
    ++acc;
    due = by_upd && R > 0 && (u0 + (uint64_t)acc) % (uint64_t)R == 0;
    // the Jastrow-field change, requested now so its loads overlap the update
    // of M^-1 (V is symmetric: row site_new across the threads is coalesced)
    constexpr int kHv = 4;
    double dv[kHv];
#pragma unroll
    for (int u = 0; u < kHv; ++u) {
      const int l = tid + u * NT;
      dv[u] = l < ns ? V[(int64_t)site_new * ns + l] - V[(int64_t)site_old * ns + l] : 0.0;
    }
    __syncthreads();   // m' and the column/row of M^-1 visible to every thread

    // v (up) or t (down): each wavefront sums a slice of the contraction
    // index for every output index, the slices are then added in order
    {
      const int j0 = (wid * n) / NW, j1 = ((wid + 1) * n) / NW;
      for (int o = lane; o < n; o += 64) {
        T s = T(0);
        if (sigma == 0)
          for (int b = j0; b < j1; ++b) s += mv[b] * Mi[b * ld + o];   // v[o], row b contiguous
        else
          for (int j = j0; j < j1; ++j) s += Mi[o * ld + j] * mv[j];   // t[o], row o of M^-1
        part[wid * n + o] = s;
      }
    }
    __syncthreads();
    for (int o = tid; o < n; o += NT) {
      T s = T(0);
#pragma unroll
      for (int w = 0; w < NW; ++w) s += part[w * n + o];
      vt[o] = s - (o == ai ? T(1) : T(0));
    }
    __syncthreads();
    // rank-1 update: up  M^-1[i][j] -= cr[i] v[j] / r;  down  M^-1[i][j] -= t[i] cr[j] / r
    const T ir = T(1.0 / r_pf);
    for (int e = tid; e < n * n; e += NT) {
      const int i = e / n, j = e - (e / n) * n;
      const T lft = sigma == 0 ? cr[i] : vt[i];
      const T rgt = sigma == 0 ? vt[j] : cr[j];
      Mi[i * ld + j] -= (lft * ir) * rgt;
    }
#pragma unroll
    for (int u = 0; u < kHv; ++u) {
      const int l = tid + u * NT;
      if (l < ns) hs[l] += dv[u];
    }
    for (int l = tid + kHv * NT; l < ns; l += NT)
      hs[l] += V[(int64_t)site_new * ns + l] - V[(int64_t)site_old * ns + l];
    for (int hh = tid; hh < M; hh += NT)
      ths[hh] += T(2) * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
    if (tid == 0) {
      pos_s[a] = Inew;
      eidx[Iold] = -1;
      eidx[Inew] = a;
      emp[sigma * ns + k] = site_old;
    }
    __syncthreads();
    } while (false);

    if (nonfinite) {
      guard1 = guard1 == kGuardPending ? kGuardFailed : kGuardPending;
      break;
    }
    ++it;
    if (due) break;
  }

  __syncthreads();
  // both non-zero blocks of X^-1: X^-1[n + i][j] = M^-1[i][j], X^-1[j][n + i] = -M^-1[i][j]
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - (e / n) * n;
    Yg[(int64_t)(n + i) * ne + j] = Mi[i * ld + j];
    Yg[(int64_t)i * ne + n + j] = -Mi[j * ld + i];
  }
  for (int b = tid; b < ne; b += NT) posg[b] = pos_s[b];
  for (int v = tid; v < n2; v += NT) empg[v] = emp[v];
  for (int l = tid; l < ns; l += NT) hg[l] = hs[l];
  for (int hh = tid; hh < M; hh += NT) thg[hh] = (double)ths[hh];
  const uint64_t n1 = n0 + (uint64_t)it;
  const bool stop = (R > 0 && (by_upd ? due : n1 % (uint64_t)R == 0)) ||
                    guard1 == kGuardPending;
  if (tid == 0) {
    P.cnt[gw] = n1;
    P.upd[gw] = u0 + (uint64_t)acc;
    P.accepted[gw] += acc;
    if (guard1 != guard0) P.guard[gw] = guard1;
    if (stop && needs_refresh) needs_refresh[gw] = 1;
  }
  return stop;
}
}  // namespace

}  // namespace mvmc
