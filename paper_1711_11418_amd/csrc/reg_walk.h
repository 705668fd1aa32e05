// Register-resident Metropolis sweep: one wavefront per walker, the non-zero
// blocks of X^-1 held in VGPRs for the whole launch, WPB walkers of one
// instance per workgroup sharing the pair-amplitude table f in LDS.
//
// With anti-parallel pairing (Eq. AP-Pf), up electrons 0..n-1 and down
// electrons n..2n-1, X = [[0, M], [-M^T, 0]] and Y = X^-1 =
// [[0, -M^-T], [M^-1, 0]]: entries of Y between two electrons of the same
// spin are zero and the hopping update keeps them zero.  Lane c < N_e keeps
// the n entries of column c in the rows of the opposite spin,
//   z[i] = Y[o_c + i][c],   o_c = n for an up electron c, 0 for a down one,
// which halves the registers and the update work of a full column.  Per
// proposal moving electron a of spin sigma (a' = a - sigma n; hopping update
// of section 3.1.2 with the fast-update ratio):
//   Y[a][c]         for c of the other spin is z_c[a'] (an indexed register
//                   move with a uniform index)
//   x'_c            the anti-parallel pair amplitude between the new
//                   spin-orbital I' and electron c: f(site', site_c) when an
//                   up electron moves and c is down, -f(site_c, site') when a
//                   down electron moves and c is up, else 0 (X_IJ = F_IJ - F_JI)
//   r_Pf            -sum_c Y[a][c] x'_c   (DPP wave reduction)
//   correlators     Gutzwiller factors, Jastrow field and v, RBM angles, all
//                   in LDS
// On acceptance, with p = -Y[a,:] (non-zero on the other spin) and
// q = -Y^T x' + e_a (non-zero on a's spin) written to the two halves of an
// LDS vector w,
//   c of a's spin:         z[i] += p_{o_c + i} q_c / r_Pf
//   c of the other spin:   z[i] -= q_{o_c + i} p_c / r_Pf
// which is Y += (p q^T - q p^T) / r_Pf restricted to its non-zero blocks.
// Every per-proposal quantity that is the same for the whole walker lives in
// scalar registers (Philox runs on the vector unit once per 64 proposals),
// so the proposal loop has no workgroup barrier.
//
// Exchange update (section 3.1.2, Fig. 5b; EXCH): up electron a (site i) and
// down electron b = n + b' (site j) trade sites; with M^-1 columns on the up
// lanes and rows on the down lanes every quantity of the rank-2 determinant
// lemma is lane-local or one wave reduction:
//   rho   = sum over down lanes of r'[b''] M^-1[b''][a]    (r' the new row a)
//   sigma = sum over up lanes of M^-1[b'][a''] c[a'']      (c the new column b)
//   t'    = M^-1 c on the down lanes (c through LDS), beta = u . t' - u[b']
//   gamma = M^-1[b'][a],  ratio D = rho sigma - beta gamma
// and on acceptance s = u^T M^-1 on the up lanes (u through LDS), then the
// Woodbury update M^-1 -= M^-1[:, a] l1^T + (t' - e_b') l2^T with
// l1 = (sigma s - beta M^-1[b', :]) / D, l2 = (rho M^-1[b', :] - gamma s) / D,
// the up lanes reading M^-1[:, a] and t' and the down lanes l1 and l2 from LDS.
//
// The workgroup-level parts (reg_load_tables, then a workgroup barrier, then
// reg_walk in every wavefront) are shared by the register-tier kernel and the
// persistent queue kernel.
#pragma once

#include "ap_block.h"
#include "common.h"
#include "wave.h"

namespace mvmc {

namespace {
using namespace wave;

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS: [f table ns x (ns+1) | Gutzwiller g per site | Jastrow v ns x ns |
// WPB x per-walker block], all tables in double (the single-precision sweep
// converts the gathered amplitudes, which equals reading a single-precision
// copy), so the proposal loop makes no global load.
__host__ __device__ inline size_t reg_table_bytes(int ns) {
  return a16((size_t)ns * (ns + 1) * sizeof(double)) + a16((size_t)ns * sizeof(double)) +
         a16((size_t)ns * ns * sizeof(double));
}
__host__ __device__ inline size_t reg_refresh_bytes(int ne_max) {
  const size_t nh = (size_t)ne_max / 2;
  return a16(nh * (nh + 1) * sizeof(double)) + a16(2 * nh * sizeof(int32_t));
}
// x' and w, each as [up half | 16-byte gap | down half] of ne_max/2 entries
__host__ __device__ inline size_t reg_half_len(int ne_max, size_t ts) {
  return (size_t)ne_max + 16 / ts;
}
__host__ __device__ inline size_t reg_walker_bytes(int ne_max, int ns, int M, size_t ts) {
  return a16(2 * reg_half_len(ne_max, ts) * ts) + a16((size_t)ns * sizeof(double)) +
         a16((size_t)M * ts) + a16((size_t)(4 * ns) * sizeof(int32_t)) +
         reg_refresh_bytes(ne_max);
}

// The n = NH register entries of a lane as groups of at most 32 dwords, the
// largest register vector the indexed-move path handles.
template <typename T, int NH>
struct RegCol {
  static constexpr int GS = NH < 128 / (int)sizeof(T) ? NH : 128 / (int)sizeof(T);
  static constexpr int NG = NH / GS;
  typedef T __attribute__((ext_vector_type(GS))) Vec;
};

// z[i] for a uniform runtime i < NH: one indexed register move per group
// (the array stays in registers), then a select between the groups.
template <typename T, int NH, typename ZArr>
__device__ __forceinline__ T pick_col(const ZArr& z, int i) {
  using RC = RegCol<T, NH>;
  static_assert(RC::NG == 1 || RC::NG == 2, "one or two register groups");
  if constexpr (RC::NG == 1) {
    return z[0][i];
  } else {
    T v0 = z[0][i & (RC::GS - 1)], v1 = z[1][i & (RC::GS - 1)];
    // keep the two extracts apart, so the select is of two values and not
    // of the two whole groups
    asm volatile("" : "+v"(v0));
    asm volatile("" : "+v"(v1));
    return i >= RC::GS ? v1 : v0;
  }
}

template <typename T> __device__ __forceinline__ const T* rbmT_ptr(const Pools& P);
template <> __device__ __forceinline__ const double* rbmT_ptr<double>(const Pools& P) { return P.rbmT64; }
template <> __device__ __forceinline__ const float* rbmT_ptr<float>(const Pools& P) { return P.rbmT32; }

// Uniform value the optimiser may not look through (keeps the compares on
// it as 32-bit scalar compares).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

}  // namespace


constexpr int kChunk = 8;   // rows per group of broadcast loads in the update

// With the in-register refresh on, register-tier walkers recompute X^-1 in
// double inside the launch at every multiple of refresh_every instead of
// stopping for the refresh kernel.
#ifndef MVMC_SWEEP_INKERNEL_REFRESH
#define MVMC_SWEEP_INKERNEL_REFRESH 1
#endif

// Double-precision recomputation inside the launch through the
// anti-parallel block (Eq. AP-Pf): the n = N_e/2 rows of M sit one per lane
// during the exchange steps (ap_steps); the final tableau then goes through
// LDS and every lane rebuilds its n entries of X^-1 = [[0, -M^-T], [M^-1, 0]]:
//   c an up electron:          z[i] = X^-1[n + i][c] = M^-1[i][c]
//   c = n + a' a down one:     z[i] = X^-1[i][c]     = -M^-1[a'][i]
// with M^-1[a][p_b] = T[p_a][b].
template <int NE_MAX, typename T, typename ZArr>
__device__ __forceinline__ int reg_refresh_ap(
    ZArr& z, int posr0,
    const double* __restrict__ fs, int ldf, int ns, int ne, int lane, double* tab,
    int32_t* piv, int32_t* pinv, double& logabs, double& sgn) {
  constexpr int NH = NE_MAX / 2;
  constexpr int LDT = NH + 1;
  using RC = RegCol<T, NH>;
  int nh = ne / 2;
  asm volatile("" : "+s"(nh));   // keep the per-index compares inside this call
  const bool live = lane < nh;
  const int su = live ? posr0 : 0;   // site of up electron `lane`
  double m[NH];
#pragma unroll
  for (int b = 0; b < NH; ++b) {
    // site of down electron b, read from its lane (no LDS round trip)
    const int sb = __builtin_amdgcn_readlane(posr0, b < nh ? nh + b : 0) - ns;
    const bool in = live && b < nh;
    const double x = fs[su * ldf + (in ? sb : 0)];
    m[b] = in ? x : 0.0;
  }
  ApState st;
  ap_steps<0, NH>(st, m, piv, lane, live, nh, 0.0);
  if (st.singular) return 1;
  logabs = st.logabs;
  sgn = st.sgn;
  if (st.parity & 1) sgn = -sgn;
  if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;   // Pf(X) = (-1)^{n(n-1)/2} det M
  if (live) {
#pragma unroll
    for (int b = 0; b < NH; ++b) tab[lane * LDT + b] = m[b];
    pinv[piv[lane]] = lane;
  }
  wave_sync();
  const bool up = lane < nh, dn = lane >= nh && lane < ne;
  // the pivot rows per column and their inverse, one entry per lane, then
  // broadcast by readlane
  const int mpiv = lane < nh ? piv[lane] : 0;
  const int mpinv = lane < nh ? pinv[lane] : 0;
  // column of T for an up lane (pinv[c]), row of T for a down lane (p_{a'},
  // fetched from lane a' by a full-wave permute)
  const int pdn = __builtin_amdgcn_ds_bpermute((dn ? lane - nh : 0) << 2, mpiv);
  const int own = up ? mpinv : (dn ? pdn : 0);
#pragma unroll
  for (int g = 0; g < RC::NG; ++g)
#pragma unroll
    for (int j = 0; j < RC::GS; ++j) {
      const int i = g * RC::GS + j;
      const int pi = __builtin_amdgcn_readlane(mpiv, i < NH ? i : 0);
      const int qi = __builtin_amdgcn_readlane(mpinv, i < NH ? i : 0);
      const double vu = tab[pi * LDT + own];
      const double vd = tab[own * LDT + qi];
      const double v = i < nh ? (up ? vu : (dn ? -vd : 0.0)) : 0.0;
      z[g][j] = (T)v;
    }
  wave_sync();
  return 0;
}

// The instance tables of a register-tier group into LDS, by every thread of
// the workgroup (WPB wavefronts); a workgroup barrier must follow before
// reg_walk reads them.
template <int WPB>
__device__ __forceinline__ void reg_load_tables(const Pools& P, const InstDev& I,
                                                unsigned char* smem) {
  const int ns = sgpr(I.ns);
  const int n2 = 2 * ns, ldf = ns + 1;
  const int64_t A_off = I.A_off, V_off = I.V_off, site_off = I.site_off;
  // shared tables: pair amplitude f[i][j] = A[i][Ns + j], Gutzwiller g,
  // Jastrow v (copies with eight loads in flight per thread)
  double* fs = (double*)smem;
  double* gs = (double*)(smem + a16((size_t)ns * ldf * sizeof(double)));
  double* vs = gs + a16((size_t)ns * sizeof(double)) / sizeof(double);
  {
    const double* A = P.A64 + A_off;
    const double* Vg = P.V + V_off;
    constexpr int U = 8;
    for (int e0 = threadIdx.x; e0 < ns * ns; e0 += 64 * WPB * U) {
      double fa[U], va[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * 64 * WPB;
        const int ec = e < ns * ns ? e : 0;
        const int i = ec / ns, j = ec - (ec / ns) * ns;
        fa[u] = A[(int64_t)i * n2 + ns + j];
        va[u] = Vg[ec];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * 64 * WPB;
        if (e < ns * ns) {
          const int i = e / ns, j = e - (e / ns) * ns;
          fs[i * ldf + j] = fa[u];
          vs[e] = va[u];
        }
      }
    }
    for (int e = threadIdx.x; e < ns; e += 64 * WPB) gs[e] = P.G[site_off + e];
  }
}

// The proposals of global walker gw (-1: none) by wavefront wv of the
// group, up to target[gw] (at most cap; without kref also only up to the
// next multiple of R).  No workgroup barrier inside.
template <typename T, int NE_MAX, int WPB, bool TRACE, bool RBM, bool EXCH>
__device__ __forceinline__ void reg_walk(const Pools& P, int gw, int wv, unsigned char* smem,
                                         int cap, uint64_t seed, TraceRec* trace,
                                         int64_t trace_cap,
                                         const uint64_t* __restrict__ trace_base,
                                         const uint64_t* __restrict__ target,
                                         int32_t* __restrict__ needs_refresh, int R, int kref,
                                         int ex64) {
  constexpr int NH = NE_MAX / 2;
  using RC = RegCol<T, NH>;
  using Vec = typename RC::Vec;
  constexpr int HD = NH + 16 / (int)sizeof(T);   // start of the down half of x' and w
  const int lane = threadIdx.x & 63;
  if (gw < 0 || P.guard[gw] == kGuardFailed) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  // instance fields read once (the loop below then holds them in registers)
  const int ns = sgpr(I.ns), ne = sgpr(I.ne), M = sgpr(I.M);
  const int nh = ne / 2;   // n_up = n_dn
  const int n2 = 2 * ns, ldf = ns + 1;
  const int64_t walker_off = I.walker_off, pos_off = I.pos_off, empty_off = I.empty_off,
                h_off = I.h_off, theta_off = I.theta_off, Y_off = I.Y_off,
                rbm_b_off = I.rbm_b_off, rbm_W_off = I.rbm_W_off, rbm_a_off = I.rbm_a_off;
  double* fs = (double*)smem;
  double* gs = (double*)(smem + a16((size_t)ns * ldf * sizeof(double)));
  double* vs = gs + a16((size_t)ns * sizeof(double)) / sizeof(double);
  const uint64_t n0 = P.cnt[gw];
  const uint64_t tg = target[gw];
  uint64_t todo = tg > n0 ? tg - n0 : 0;
  if (todo > (uint64_t)cap) todo = (uint64_t)cap;
  if (R > 0 && !kref) {
    const uint64_t left = (uint64_t)R - n0 % (uint64_t)R;
    if (todo > left) todo = left;
  }
  if (todo == 0) return;
  const int n_prop = (int)todo;
  const int64_t lw = gw - walker_off;

  unsigned char* q = smem + reg_table_bytes(ns) +
                     (size_t)wv * reg_walker_bytes(NE_MAX, ns, M, sizeof(T));
  T* xn = (T*)q;                               // x', halves at 0 and HD
  T* w = xn + reg_half_len(NE_MAX, sizeof(T));  // p and q, halves at 0 and HD
  q += a16(2 * reg_half_len(NE_MAX, sizeof(T)) * sizeof(T));
  double* hs = (double*)q;
  q += a16((size_t)ns * sizeof(double));
  T* ths = (T*)q;
  q += a16((size_t)M * sizeof(T));
  int32_t* eidx = (int32_t*)q;      // 2ns
  int32_t* emp = eidx + n2;         // 2ns
  q += a16((size_t)(4 * ns) * sizeof(int32_t));
  // refresh scratch: tableau, pivot rows per column and inverse
  double* tab = (double*)q;
  q += a16((size_t)NH * (NH + 1) * sizeof(double));
  int32_t* piv = (int32_t*)q;
  int32_t* pinv = piv + NH;

  int32_t* posg = P.pos + pos_off + lw * ne;
  int32_t* empg = P.empty + empty_off + lw * n2;
  double* hg = P.h + h_off + lw * ns;
  double* thg = P.theta + theta_off + lw * M;
  T* Yg = (T*)P.Y + Y_off + lw * ne * ne;

  const bool live = lane < ne;
  const bool lane_up = lane < nh;
  const int slot = lane_up ? lane : HD + (lane - nh);   // lane's entry of x' and w
  const T* wl = w + (lane_up ? HD : 0);                 // the half of w the lane's rows read
  const T* xl = xn + (lane_up ? HD : 0);                // the same half of x'
  const int rb = lane_up ? nh : 0;                      // first row of the lane's entries

  for (int v = lane; v < n2; v += 64) {
    eidx[v] = -1;
    emp[v] = empg[v];
  }
  for (int l = lane; l < ns; l += 64) hs[l] = hg[l];
  for (int hh = lane; hh < M; hh += 64) ths[hh] = (T)thg[hh];
  for (int c = lane; c < 2 * (int)reg_half_len(NE_MAX, sizeof(T)); c += 64) xn[c] = T(0);
  int posr = live ? posg[lane] : -1;
  wave_sync();
  if (posr >= 0) eidx[posr] = lane;

  Vec z[RC::NG];
  {
    const int lc = live ? lane : 0;
#pragma unroll
    for (int g = 0; g < RC::NG; ++g)
#pragma unroll
      for (int j = 0; j < RC::GS; ++j) {
        const int i = g * RC::GS + j;
        const int ic = i < nh ? i : 0;   // clamped row: every load in bounds
        const T v = Yg[(size_t)(rb + ic) * ne + lc];
        z[g][j] = (live && i < nh) ? v : T(0);
      }
  }
  wave_sync();

  const T* raT = rbmT_ptr<T>(P) + rbm_a_off;                 // a (2Ns)
  const T* WT = rbmT_ptr<T>(P) + rbm_W_off;                  // W^T [2Ns][M]
  const uint64_t tb = TRACE ? trace_base[gw] : 0;
  const int nemp = ns - nh;   // empty sites of either spin
  int64_t acc = 0;
  int singular = 0;
  double last_logpf = 0.0, last_sgn = 0.0;
  bool refreshed = false;
  const double* rbT64 = P.rbmT64;

  // proposals (or applied updates) until the next refresh
  const bool by_upd = P.refresh_upd != 0;
  const uint64_t u0 = P.upd[gw];
  int to_refresh = R > 0 ? R - (int)((by_upd ? u0 : n0) % (uint64_t)R) : 0;
  // Philox words of the next 64 proposals, one proposal per lane: the vector
  // unit evaluates them together and each proposal reads its four words back
  uint32_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
  // A ratio that is not finite (NaN or Inf) refreshes X^-1 in double at once
  // and the same proposal is tried again; not finite a second time, the
  // walker stops there (guard word kGuardFailed, reported by the host).
  bool tripped = false, failed = false;
  int it = 0;   // proposals taken so far
  int batch = -1;
  while (it < n_prop) {
    const uint64_t n = n0 + (uint64_t)it;
    const int64_t acc_before = acc;
    const int rs = it & 63;
    if ((it >> 6) != batch) {
      batch = it >> 6;
      const uint4 d = draw(seed, n + (uint64_t)lane, (uint32_t)gw, 0u);
      d0 = d.x;
      d1 = d.y;
      d2 = d.z;
      d3 = d.w;
    }
    bool nonfinite = false;
    do {
    uint4 r;
    r.x = (uint32_t)__builtin_amdgcn_readlane((int)d0, rs);
    r.y = (uint32_t)__builtin_amdgcn_readlane((int)d1, rs);
    r.z = (uint32_t)__builtin_amdgcn_readlane((int)d2, rs);
    r.w = (uint32_t)__builtin_amdgcn_readlane((int)d3, rs);
    if (EXCH && (int)(r.w & 63u) < ex64) {
      // ---------------------------------------------------- exchange
      const int a = opaque(sgpr(scaled(r.x, nh)));
      const int bd = opaque(sgpr(scaled(r.y, nh)));
      const int b = nh + bd;
      const int si = sgpr(__builtin_amdgcn_readlane(posr, a));
      const int sj = sgpr(__builtin_amdgcn_readlane(posr, b)) - ns;
      if (si == sj || eidx[sj] >= 0 || eidx[si + ns] >= 0) {   // no such move
        if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
          TraceRec rec;
          rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
          rec.ratio = 0.0; rec.b = b; rec.pad = 0;
          trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
        }
        break;
      }
      const T ya = pick_col<T, NH>(z, a);    // down lane b'': -M^-1[b''][a]
      const T yb = pick_col<T, NH>(z, bd);   // up lane a'':   M^-1[b'][a'']
      const bool dnl = live && !lane_up;
      const int sl = live ? posr - (lane_up ? 0 : ns) : 0;   // site of the lane's electron
      // down lanes: new row a of M and its change; up lanes: new column b off row a
      const double fnew = lane == b ? fs[sj * ldf + si] : fs[sj * ldf + sl];
      const double fold = fs[si * ldf + sl];
      const double fcol = lane == a ? fs[si * ldf + sj] : fs[sl * ldf + si];
      const T rn = dnl ? (T)fnew : T(0);
      const T uu = dnl ? (T)(fnew - fold) : T(0);
      const T cv = lane_up ? (T)fcol : T(0);
      if (live) {
        xn[slot] = lane_up ? cv : T(0);
        w[slot] = lane_up ? T(0) : uu;
      }
      double pr = (double)(rn * -ya), ps = (double)(yb * cv);
      double rbm = 0.0;
      if (RBM && M) {
        for (int hh = lane; hh < M; hh += 64) {
          const T d = T(2) * (WT[(int64_t)sj * M + hh] - WT[(int64_t)si * M + hh] +
                              WT[(int64_t)(si + ns) * M + hh] - WT[(int64_t)(sj + ns) * M + hh]);
          const T th = ths[hh];
          rbm += (double)(log2cosh(th + d) - log2cosh(th));
        }
        rbm = wave_total(rbm);
      }
      const double rho = wave_total(pr), sig = wave_total(ps);
      const int ylo = __builtin_amdgcn_readlane(__double2loint((double)yb), a);
      const int yhi = __builtin_amdgcn_readlane(__double2hiint((double)yb), a);
      const double gam = __hiloint2double(yhi, ylo);
      wave_sync();   // c on the up half of x' for every lane
      // t'[b''] = sum_a'' M^-1[b''][a''] c[a''] on the down lanes (x' up half)
      T tc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int g = 0; g < RC::NG; ++g)
#pragma unroll
        for (int j0 = 0; j0 < RC::GS; j0 += kChunk) {
#pragma unroll
          for (int j = j0; j < j0 + kChunk && j < RC::GS; ++j)
            tc[j & 3] += z[g][j] * xn[g * RC::GS + j];
          asm volatile("" ::: "memory");
        }
      const T tp = dnl ? -((tc[0] + tc[1]) + (tc[2] + tc[3])) : T(0);
      const double ub = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint((double)uu), b),
                                         __builtin_amdgcn_readlane(__double2loint((double)uu), b));
      const double bet = wave_total((double)(uu * tp)) - ub;
      const double Dd = rho * sig - bet * gam;
      double logc = 0.0;
      if (RBM && M)
        logc = 2.0 * ((double)raT[sj] - (double)raT[si] + (double)raT[si + ns] -
                      (double)raT[sj + ns]) + rbm;
      const double Rt = Dd * exp(logc);
      if (!isfinite(Rt)) {
        nonfinite = true;
        break;
      }
      const int accept = sgpr(uniform53(r.z, r.w) < Rt * Rt ? 1 : 0);
      if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = sj; rec.accepted = accept;
        rec.ratio = Rt; rec.b = b; rec.pad = 0;
        trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
      }
      if (!accept) break;
      ++acc;
      // s[a''] = sum_b'' u[b''] M^-1[b''][a''] on the up lanes (u on the down half of w)
      T sc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int g = 0; g < RC::NG; ++g)
#pragma unroll
        for (int j0 = 0; j0 < RC::GS; j0 += kChunk) {
#pragma unroll
          for (int j = j0; j < j0 + kChunk && j < RC::GS; ++j)
            sc[j & 3] += z[g][j] * w[HD + g * RC::GS + j];
          asm volatile("" ::: "memory");
        }
      const double sv = (double)((sc[0] + sc[1]) + (sc[2] + sc[3]));
      const double iD = 1.0 / Dd;
      // up lanes: l1, l2; down lanes: M^-1[b''][a] and t' - e_b'
      const T l1 = (T)((sig * sv - bet * (double)yb) * iD);
      const T l2 = (T)((rho * (double)yb - gam * sv) * iD);
      const T cav = -ya;
      const T tv = tp - (lane == b ? T(1) : T(0));
      wave_sync();   // every read of c and u done
      if (live) {
        xn[slot] = lane_up ? l1 : cav;
        w[slot] = lane_up ? l2 : tv;
      }
      wave_sync();
      // up lanes (column of M^-1):  z -= M^-1[:, a] l1 + t l2
      // down lanes (-row of M^-1):  z += M^-1[b'', a] l1 + t[b''] l2
      const T ka = lane_up ? -l1 : cav;
      const T kb = lane_up ? -l2 : tv;
#pragma unroll
      for (int g = 0; g < RC::NG; ++g)
#pragma unroll
        for (int j0 = 0; j0 < RC::GS; j0 += kChunk) {
#pragma unroll
          for (int j = j0; j < j0 + kChunk && j < RC::GS; ++j)
            z[g][j] += xl[g * RC::GS + j] * ka + wl[g * RC::GS + j] * kb;
          asm volatile("" ::: "memory");
        }
      // the list slots of j (up list) and i (down list)
      int kup = -1, kdn = -1;
      for (int c0 = 0; c0 < ns; c0 += 64) {
        const int idx = c0 + lane;
        const uint64_t mu = __ballot(idx < ns && emp[idx] == sj);
        const uint64_t md = __ballot(idx < ns && emp[ns + idx] == si);
        if (mu) kup = c0 + __builtin_ctzll(mu);
        if (md) kdn = c0 + __builtin_ctzll(md);
      }
      if (RBM)
        for (int hh = lane; hh < M; hh += 64)
          ths[hh] += T(2) * (WT[(int64_t)sj * M + hh] - WT[(int64_t)si * M + hh] +
                             WT[(int64_t)(si + ns) * M + hh] - WT[(int64_t)(sj + ns) * M + hh]);
      if (lane == a) posr = sj;
      if (lane == b) posr = si + ns;
      if (lane == 0) {
        eidx[si] = -1;
        eidx[sj + ns] = -1;
        eidx[sj] = a;
        eidx[si + ns] = b;
        emp[kup] = si;
        emp[ns + kdn] = sj;
      }
      wave_sync();
      break;
    }
    const int a = opaque(sgpr(scaled(r.x, ne)));
    const int sigma = a >= nh ? 1 : 0;
    if (nemp == 0) {
      if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.b = -1; rec.pad = 0;
        rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
        rec.ratio = 0.0;
        trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
      }
      break;
    }
    const int kk_emp = sgpr(scaled(r.y, nemp));
    const int site_new = sgpr(emp[sigma * ns + kk_emp]);
    const int Inew = site_new + sigma * ns;
    const int Iold = sgpr(__builtin_amdgcn_readlane(posr, a));
    const int site_old = Iold - sigma * ns;
    const int ai = opaque(a - sigma * nh);

    // this lane's electron is of the other spin than a: its x'_c may be non-zero
    const bool oppl = live && (lane_up == (sigma != 0));
    const T ya = pick_col<T, NH>(z, ai);
    const int sp = live ? posr - (lane_up ? 0 : ns) : 0;   // site of the lane's electron
    const double fv = fs[sigma ? sp * ldf + site_new : site_new * ldf + sp];
    const T xb = oppl ? (T)(sigma ? -fv : fv) : T(0);
    if (live) xn[slot] = xb;
    double part = (double)(ya * xb);
    double rbm = 0.0;
    if (RBM && M) {
      for (int hh = lane; hh < M; hh += 64) {
        const T d = T(2) * (WT[(int64_t)Inew * M + hh] - WT[(int64_t)Iold * M + hh]);
        const T th = ths[hh];
        rbm += (double)(log2cosh(th + d) - log2cosh(th));
      }
      rbm = wave_total(rbm);
    }
    const double r_pf = -wave_total(part);
    const int opp = (1 - sigma) * ns;
    double logc = gs[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  gs[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                  hs[site_old] - vs[site_old * ns + site_new];
    if (RBM && M) logc += 2.0 * ((double)raT[Inew] - (double)raT[Iold]) + rbm;
    const double Rt = r_pf * exp(logc);
    if (!isfinite(Rt)) {
      nonfinite = true;
      break;
    }
    const double u = uniform53(r.z, r.w);
    const int accept = sgpr(u < Rt * Rt ? 1 : 0);
    if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
      TraceRec rec;
      rec.b = -1; rec.pad = 0;
      rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = Inew; rec.accepted = accept;
      rec.ratio = Rt;
      trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
    }
    if (!accept) break;
    ++acc;
    wave_sync();   // x' of every lane visible

    // q_c = -sum_j Y[j][c] x'_j + delta_{c,a} on a's spin (j over the other
    // spin, the half of x' at hq); p_c = -Y[a][c] on the other spin
    const bool same = live && !oppl;
    const int hq = sigma ? 0 : HD;
    T sc[4] = {T(0), T(0), T(0), T(0)};   // four independent FMA chains
#pragma unroll
    for (int g = 0; g < RC::NG; ++g)
#pragma unroll
      for (int j0 = 0; j0 < RC::GS; j0 += kChunk) {
#pragma unroll
        for (int j = j0; j < j0 + kChunk && j < RC::GS; ++j)
          sc[j & 3] += z[g][j] * xn[hq + g * RC::GS + j];
        asm volatile("" ::: "memory");   // bound the number of broadcast loads in flight
      }
    const T sq = (sc[0] + sc[1]) + (sc[2] + sc[3]);
    const T qc = same ? (lane == a ? T(1) : T(0)) - sq : T(0);
    const T pc = oppl ? -ya : T(0);
    if (live) w[slot] = same ? qc : pc;
    wave_sync();
    const T ir = T(1.0 / r_pf);
    const T coef = same ? qc * ir : -(pc * ir);
#pragma unroll
    for (int g = 0; g < RC::NG; ++g)
#pragma unroll
      for (int j0 = 0; j0 < RC::GS; j0 += kChunk) {
#pragma unroll
        for (int j = j0; j < j0 + kChunk && j < RC::GS; ++j)
          z[g][j] += wl[g * RC::GS + j] * coef;
        asm volatile("" ::: "memory");
      }
    for (int l = lane; l < ns; l += 64) hs[l] += vs[site_new * ns + l] - vs[site_old * ns + l];
    if (RBM)
      for (int hh = lane; hh < M; hh += 64)
        ths[hh] += T(2) * (WT[(int64_t)Inew * M + hh] - WT[(int64_t)Iold * M + hh]);
    if (lane == a) posr = Inew;
    if (lane == 0) {
      eidx[Iold] = -1;
      eidx[Inew] = a;
      emp[sigma * ns + kk_emp] = site_old;
    }
    wave_sync();
    } while (false);

    bool do_refresh = false;
    if (nonfinite) {
      if (tripped) {
        failed = true;
        break;
      }
      tripped = true;
      do_refresh = true;   // the proposal is tried again after the refresh
    } else {
      tripped = false;
      ++it;
      bool wrapped = false;
      if (R > 0 && (!by_upd || acc != acc_before) && --to_refresh == 0) {
        to_refresh = R;
        wrapped = true;
      }
#if MVMC_SWEEP_INKERNEL_REFRESH
      // periodic double-precision recomputation, inside the launch
      do_refresh = kref && wrapped;
#endif
    }
    if (do_refresh) {
      double lp, sg;
      singular = reg_refresh_ap<NE_MAX, T>(z, posr, fs, ldf, ns, ne, lane, tab, piv, pinv,
                                           lp, sg);
      last_logpf = lp;
      last_sgn = sg;
      refreshed = true;
      // Jastrow field and RBM angles from scratch (v is symmetric: row mm
      // of v read across the lanes)
      for (int l = lane; l < ns; l += 64) {
        double sum = 0.0;
#pragma unroll 8
        for (int mm = 0; mm < ns; ++mm)
          sum += vs[mm * ns + l] *
                 (double)((eidx[mm] >= 0 ? 1 : 0) + (eidx[mm + ns] >= 0 ? 1 : 0) - 1);
        hs[l] = sum;
      }
      if (RBM)
      for (int hh = lane; hh < M; hh += 64) {
        double th = rbT64[rbm_b_off + hh];
        for (int v = 0; v < n2; ++v)
          th += rbT64[rbm_W_off + (int64_t)v * M + hh] * (eidx[v] >= 0 ? 1.0 : -1.0);
        ths[hh] = (T)th;
      }
      wave_sync();
      if (singular) break;
    }
  }

  // write the walker back (the same-spin blocks of Y stay zero in memory)
  if (live) posg[lane] = posr;
#pragma unroll
  for (int g = 0; g < RC::NG; ++g)
#pragma unroll
    for (int j = 0; j < RC::GS; ++j) {
      const int i = g * RC::GS + j;
      if (live && i < nh) Yg[(size_t)(rb + i) * ne + lane] = z[g][j];
    }
  for (int v = lane; v < n2; v += 64) empg[v] = emp[v];
  for (int l = lane; l < ns; l += 64) hg[l] = hs[l];
  for (int hh = lane; hh < M; hh += 64) thg[hh] = (double)ths[hh];
  if (lane == 0) {
    const uint64_t n1 = n0 + (uint64_t)it;
    P.cnt[gw] = n1;
    P.upd[gw] = u0 + (uint64_t)acc;
    P.accepted[gw] += acc;
    if (failed) P.guard[gw] = kGuardFailed;
    if (R > 0 && !kref && n1 % (uint64_t)R == 0) needs_refresh[gw] = 1;
    if (refreshed) {
      P.logpf[gw] = singular ? -INFINITY : last_logpf;
      P.sgnpf[gw] = singular ? 0.0 : last_sgn;
      P.status[gw] = singular;
    }
  }
}

}  // namespace mvmc
