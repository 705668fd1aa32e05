// Register-resident Metropolis sweep: one wavefront per walker, X^-1 held in
// VGPRs for the whole launch, WPB walkers of one instance per workgroup
// sharing the pair-amplitude table f in LDS.
//
// Lane l owns the columns c = l + 64k (k < KC) of Y = X^-1 and keeps
// y[k][i] = Y[i][c] for every row i.  Per proposal (same arithmetic as the
// LDS kernel; hopping update of section 3.1.2 with the fast-update ratio):
//   row a of Y      y[k][a], a uniform index (branch tree over a)
//   x'_c            the anti-parallel pair amplitude between the new
//                   spin-orbital I' and electron c: f(site', site_c) when an
//                   up electron moves and c is down, -f(site_c, site') when a
//                   down electron moves and c is up, else 0 (Eq. AP-Pf with
//                   X_IJ = F_IJ - F_JI)
//   r_Pf            -sum_c Y[a][c] x'_c   (DPP wave reduction)
//   correlators     scalar loads (Gutzwiller, Jastrow field in LDS, RBM)
// On acceptance, with p = -Y[a,:], q = -Y^T x' + e_a (column sums over the
// registers with x' broadcast from LDS):
//   y[k][i] += p_i (q_c / r_Pf) - q_i (p_c / r_Pf)
// Every per-proposal quantity that is the same for the whole walker lives in
// scalar registers (Philox runs on the scalar unit), so the proposal loop has
// no workgroup barrier.
#include "ap_block.h"
#include "launch.h"
#include "wave.h"

namespace mvmc {

namespace {
using namespace wave;

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS: [f table ns x (ns+1) in double | WPB x per-walker block]; the
// single-precision sweep converts the gathered amplitudes, which equals
// reading the single-precision copy of the table.
__host__ __device__ inline size_t reg_table_bytes(int ns, size_t ts) {
  (void)ts;
  return a16((size_t)ns * (ns + 1) * sizeof(double));
}
__host__ __device__ inline size_t reg_refresh_bytes(int ne_max) {
  const size_t nh = (size_t)ne_max / 2;
  return a16(nh * (nh + 1) * sizeof(double)) + a16(nh * sizeof(double)) +
         a16(2 * nh * sizeof(int32_t));
}
__host__ __device__ inline size_t reg_walker_bytes(int ne_max, int ns, int M, size_t ts) {
  return a16(3 * (size_t)ne_max * ts) + a16((size_t)ns * sizeof(double)) + a16((size_t)M * ts) +
         a16((size_t)(4 * ns + ne_max) * sizeof(int32_t)) + reg_refresh_bytes(ne_max);
}

// y[a] for a uniform runtime index a, as a branch tree over compile-time
// indices.  The empty volatile asm in each leaf keeps the compiler from
// folding the tree back into one dynamically indexed access, which would
// move the whole register array to scratch memory.
template <typename T, int N, int LO, int HI>
__device__ __forceinline__ T pick(const T (&y)[N], int a) {
  if constexpr (HI - LO == 1) {
    asm volatile("" ::: );
    return y[LO];
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (a < MID) return pick<T, N, LO, MID>(y, a);
    return pick<T, N, MID, HI>(y, a);
  }
}

template <typename T> __device__ __forceinline__ const T* rbmT_ptr(const Pools& P);
template <> __device__ __forceinline__ const double* rbmT_ptr<double>(const Pools& P) { return P.rbmT64; }
template <> __device__ __forceinline__ const float* rbmT_ptr<float>(const Pools& P) { return P.rbmT32; }

// Uniform value the optimiser may not look through (keeps branch-tree tests
// as 32-bit scalar compares).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

}  // namespace

size_t sweep_reg_lds_bytes(int ne_max, int ns, int M, size_t tsize, int wpb) {
  return reg_table_bytes(ns, tsize) + (size_t)wpb * reg_walker_bytes(ne_max, ns, M, tsize);
}

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
// LDS and every lane rebuilds its column c of X^-1 = [[0, -M^-T], [M^-1, 0]]:
//   c an up electron:          X^-1[n + a][c] = M^-1[a][c]
//   c = n + a' a down one:     X^-1[q][c]     = -M^-1[a'][q]
// with M^-1[a][p_b] = T[p_a][b]; same-spin blocks are zero.
template <int NE_MAX, typename T>
__device__ __forceinline__ int reg_refresh_ap(T (&y)[1][NE_MAX], int posr0,
                                              const double* __restrict__ fs, int ldf, int ns,
                                              int ne, int lane, int32_t* posl, double* tab,
                                              double* rowp, int32_t* piv, int32_t* pinv,
                                              double& logabs, double& sgn) {
  constexpr int NH = NE_MAX / 2;
  constexpr int LDT = NH + 1;
  int nh = ne / 2;
  asm volatile("" : "+s"(nh));   // keep the per-index compares inside this call
  if (lane < NE_MAX) posl[lane] = posr0;
  wave_sync();
  const bool live = lane < nh;
  const int su = live ? posr0 : 0;   // site of up electron `lane`
  double m[NH];
#pragma unroll
  for (int b = 0; b < NH; ++b) {
    const bool in = live && b < nh;
    const int sd = in ? posl[nh + b] - ns : 0;
    m[b] = in ? fs[su * ldf + sd] : 0.0;
  }
  ApState st;
  ap_steps<0, NH>(st, m, rowp, piv, lane, live, nh, 0.0);
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
  // column of T for an up lane (pinv[c]), row of T for a down lane (p_{a'})
  const int own = up ? pinv[lane] : (dn ? piv[lane - nh] : 0);
#pragma unroll
  for (int r = 0; r < NE_MAX; ++r) {
    double v = 0.0;
    if (up && r >= nh && r < ne) v = tab[piv[r >= nh ? r - nh : 0] * LDT + own];
    else if (dn && r < nh) v = -tab[own * LDT + pinv[r < nh ? r : 0]];
    y[0][r] = (T)v;
  }
  wave_sync();
  return 0;
}

template <typename T, int NE_MAX, int WPB, bool TRACE, bool RBM>
__global__ __launch_bounds__(64 * WPB) void k_sweep_reg(Pools P, const int32_t* __restrict__ wlist,
                                                        int cap, uint64_t seed, TraceRec* trace,
                                                        int64_t trace_cap,
                                                        const uint64_t* __restrict__ trace_base,
                                                        const uint64_t* __restrict__ target,
                                                        int32_t* __restrict__ needs_refresh, int R,
                                                        int kref) {
  constexpr int KC = (NE_MAX + 63) / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = sgpr(threadIdx.x >> 6);
  const int g0 = wlist[blockIdx.x * WPB];
  const InstDev& I = P.inst[P.walker_inst[g0]];
  const int ns = I.ns, ne = I.ne, n2 = 2 * ns, M = I.M, nup = I.nup;
  const int ldf = ns + 1;

  // shared pair-amplitude table f[i][j] = A[i][Ns + j]
  double* fs = (double*)smem;
  {
    const double* A = P.A64 + I.A_off;
    for (int e = threadIdx.x; e < ns * ns; e += 64 * WPB) {
      const int i = e / ns, j = e - (e / ns) * ns;
      fs[i * ldf + j] = A[(int64_t)i * n2 + ns + j];
    }
  }
  __syncthreads();   // the only workgroup barrier

  const int gw = sgpr(wlist[blockIdx.x * WPB + wv]);
  if (gw < 0) return;
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
  const int64_t lw = gw - I.walker_off;

  unsigned char* q = smem + reg_table_bytes(ns, sizeof(T)) +
                     (size_t)wv * reg_walker_bytes(NE_MAX, ns, M, sizeof(T));
  T* xn = (T*)q;
  T* pv = xn + NE_MAX;
  T* qv = pv + NE_MAX;
  q += a16(3 * (size_t)NE_MAX * sizeof(T));
  double* hs = (double*)q;
  q += a16((size_t)ns * sizeof(double));
  T* ths = (T*)q;
  q += a16((size_t)M * sizeof(T));
  int32_t* eidx = (int32_t*)q;      // 2ns
  int32_t* emp = eidx + n2;         // 2ns
  int32_t* posl = emp + n2;         // NE_MAX: configuration broadcast for the refresh
  q += a16((size_t)(4 * ns + NE_MAX) * sizeof(int32_t));
  // refresh scratch: tableau, pivot row, pivot rows per column and inverse
  double* tab = (double*)q;
  q += a16((size_t)(NE_MAX / 2) * (NE_MAX / 2 + 1) * sizeof(double));
  double* rowp = (double*)q;
  q += a16((size_t)(NE_MAX / 2) * sizeof(double));
  int32_t* piv = (int32_t*)q;
  int32_t* pinv = piv + NE_MAX / 2;

  int32_t* posg = P.pos + I.pos_off + lw * ne;
  int32_t* empg = P.empty + I.empty_off + lw * n2;
  double* hg = P.h + I.h_off + lw * ns;
  double* thg = P.theta + I.theta_off + lw * M;
  T* Yg = (T*)P.Y + I.Y_off + lw * ne * ne;

  for (int v = lane; v < n2; v += 64) {
    eidx[v] = -1;
    emp[v] = empg[v];
  }
  for (int l = lane; l < ns; l += 64) hs[l] = hg[l];
  for (int hh = lane; hh < M; hh += 64) ths[hh] = (T)thg[hh];
  for (int c = lane; c < 3 * NE_MAX; c += 64) xn[c] = T(0);
  int posr[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = lane + 64 * k;
    posr[k] = c < ne ? posg[c] : -1;
  }
  wave_sync();
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (posr[k] >= 0) eidx[posr[k]] = lane + 64 * k;

  T y[KC][NE_MAX];
#pragma unroll
  for (int i = 0; i < NE_MAX; ++i) {
    const T* row = Yg + (size_t)(i < ne ? i : 0) * ne;   // uniform row pointer
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int c = lane + 64 * k;
      y[k][i] = (c < ne && i < ne) ? row[c] : T(0);
    }
  }
  wave_sync();

  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const T* raT = rbmT_ptr<T>(P) + I.rbm_a_off;                 // a (2Ns)
  const T* WT = rbmT_ptr<T>(P) + I.rbm_W_off;                  // W^T [2Ns][M]
  const uint64_t tb = TRACE ? trace_base[gw] : 0;
  int64_t acc = 0;
  int singular = 0;
  double last_logpf = 0.0, last_sgn = 0.0;
  bool refreshed = false;
  const double* rbT64 = P.rbmT64;

  int to_refresh = R > 0 ? R - (int)(n0 % (uint64_t)R) : 0;   // proposals until the next refresh
  // Philox words of the next 64 proposals, one proposal per lane: the vector
  // unit evaluates them together and each proposal reads its four words back
  uint32_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
  for (int it = 0; it < n_prop; ++it) {
    const uint64_t n = n0 + (uint64_t)it;
    const int slot = it & 63;
    if (slot == 0) {
      const uint4 d = draw(seed, n + (uint64_t)lane, (uint32_t)gw, 0u);
      d0 = d.x;
      d1 = d.y;
      d2 = d.z;
      d3 = d.w;
    }
    do {
    uint4 r;
    r.x = (uint32_t)__builtin_amdgcn_readlane((int)d0, slot);
    r.y = (uint32_t)__builtin_amdgcn_readlane((int)d1, slot);
    r.z = (uint32_t)__builtin_amdgcn_readlane((int)d2, slot);
    r.w = (uint32_t)__builtin_amdgcn_readlane((int)d3, slot);
    const int a = opaque(sgpr(scaled(r.x, ne)));
    const int sigma = a >= nup ? 1 : 0;
    const int nemp = ns - (sigma ? I.ndn : nup);
    if (nemp == 0) {
      if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
        rec.ratio = 0.0;
        trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
      }
      break;
    }
    const int kk_emp = sgpr(scaled(r.y, nemp));
    const int site_new = sgpr(emp[sigma * ns + kk_emp]);
    const int Inew = site_new + sigma * ns;
    const int ka = a >> 6, la = a & 63;
    int pa = posr[0];
#pragma unroll
    for (int k = 1; k < KC; ++k)
      if (ka == k) pa = posr[k];
    const int Iold = sgpr(__builtin_amdgcn_readlane(pa, la));
    const int site_old = Iold - sigma * ns;

    // correlator terms: scalar loads issued before the vector work
    const int opp = (1 - sigma) * ns;
    const double gnew = G[site_new], gold = G[site_old];
    const double vio = V[(int64_t)site_old * ns + site_new];

    T ya[KC], xc[KC];
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      ya[k] = pick<T, NE_MAX, 0, NE_MAX>(y[k], a);
      const int c = lane + 64 * k;
      const int pb = posr[k];
      T xb = T(0);
      if (c < ne && c != a) {
        if (sigma == 0) {
          if (pb >= ns) xb = (T)fs[site_new * ldf + (pb - ns)];
        } else {
          if (pb < ns) xb = -(T)fs[pb * ldf + site_new];
        }
      }
      xc[k] = xb;
      if (c < NE_MAX) xn[c] = xb;
      part += (double)(ya[k] * xb);
    }
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
    double logc = gnew * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  gold * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] - hs[site_old] -
                  vio;
    if (RBM && M) logc += 2.0 * ((double)raT[Inew] - (double)raT[Iold]) + rbm;
    const double Rt = r_pf * exp(logc);
    const double u = uniform53(r.z, r.w);
    const int accept = sgpr(u < Rt * Rt ? 1 : 0);
    if (TRACE && lane == 0 && n - tb < (uint64_t)trace_cap) {
      TraceRec rec;
      rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = Inew; rec.accepted = accept;
      rec.ratio = Rt;
      trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
    }
    if (!accept) break;
    ++acc;
    wave_sync();   // x' of every lane visible

    // q_c = -sum_j Y[j][c] x'_j + delta_{c,a};  p_c = -Y[a][c]
    T pc[KC], qc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      T s = T(0);
#pragma unroll
      for (int j0 = 0; j0 < NE_MAX; j0 += kChunk) {
#pragma unroll
        for (int j = j0; j < j0 + kChunk && j < NE_MAX; ++j) s += y[k][j] * xn[j];
        asm volatile("" ::: "memory");   // bound the number of broadcast loads in flight
      }
      const int c = lane + 64 * k;
      qc[k] = (c == a ? T(1) : T(0)) - s;
      pc[k] = -ya[k];
      if (c < NE_MAX) {
        pv[c] = pc[k];
        qv[c] = qc[k];
      }
    }
    wave_sync();
    const T ir = T(1.0 / r_pf);
#pragma unroll
    for (int i0 = 0; i0 < NE_MAX; i0 += kChunk) {
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const T qs = qc[k] * ir, ps = pc[k] * ir;
#pragma unroll
        for (int i = i0; i < i0 + kChunk && i < NE_MAX; ++i) y[k][i] += pv[i] * qs - qv[i] * ps;
      }
      asm volatile("" ::: "memory");
    }
    for (int l = lane; l < ns; l += 64)
      hs[l] += V[(int64_t)site_new * ns + l] - V[(int64_t)site_old * ns + l];
    if (RBM)
      for (int hh = lane; hh < M; hh += 64)
        ths[hh] += T(2) * (WT[(int64_t)Inew * M + hh] - WT[(int64_t)Iold * M + hh]);
#pragma unroll
    for (int k = 0; k < KC; ++k)
      if (ka == k && lane == la) posr[k] = Inew;
    if (lane == 0) {
      eidx[Iold] = -1;
      eidx[Inew] = a;
      emp[sigma * ns + kk_emp] = site_old;
    }
    wave_sync();
    } while (false);

    // periodic double-precision recomputation, inside the launch
#if MVMC_SWEEP_INKERNEL_REFRESH
    if (R > 0 && --to_refresh == 0) to_refresh = R;
    if (kref && R > 0 && to_refresh == R) {
      double lp, sg;
      static_assert(KC == 1, "register tiers hold one column per lane");
      singular = reg_refresh_ap<NE_MAX, T>(y, posr[0], fs, ldf, ns, ne, lane, posl, tab, rowp,
                                           piv, pinv, lp, sg);
      last_logpf = lp;
      last_sgn = sg;
      refreshed = true;
      // Jastrow field and RBM angles from scratch (V is symmetric: row mm of
      // V read across the lanes is coalesced)
      for (int l = lane; l < ns; l += 64) {
        double sum = 0.0;
#pragma unroll 8
        for (int mm = 0; mm < ns; ++mm)
          sum += V[(int64_t)mm * ns + l] *
                 (double)((eidx[mm] >= 0 ? 1 : 0) + (eidx[mm + ns] >= 0 ? 1 : 0) - 1);
        hs[l] = sum;
      }
      if (RBM)
      for (int hh = lane; hh < M; hh += 64) {
        double th = rbT64[I.rbm_b_off + hh];
        for (int v = 0; v < n2; ++v)
          th += rbT64[I.rbm_W_off + (int64_t)v * M + hh] * (eidx[v] >= 0 ? 1.0 : -1.0);
        ths[hh] = (T)th;
      }
      wave_sync();
      if (singular) break;
    }
#endif
  }

  // write the walker back
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = lane + 64 * k;
    if (c < ne) posg[c] = posr[k];
  }
#pragma unroll
  for (int i = 0; i < NE_MAX; ++i) {
    if (i < ne) {
      T* row = Yg + (size_t)i * ne;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int c = lane + 64 * k;
        if (c < ne) row[c] = y[k][i];
      }
    }
  }
  for (int v = lane; v < n2; v += 64) empg[v] = emp[v];
  for (int l = lane; l < ns; l += 64) hg[l] = hs[l];
  for (int hh = lane; hh < M; hh += 64) thg[hh] = (double)ths[hh];
  if (lane == 0) {
    const uint64_t n1 = n0 + (uint64_t)n_prop;
    P.cnt[gw] = n1;
    P.accepted[gw] += acc;
    if (R > 0 && !kref && n1 % (uint64_t)R == 0) needs_refresh[gw] = 1;
    if (refreshed) {
      P.logpf[gw] = singular ? -INFINITY : last_logpf;
      P.sgnpf[gw] = singular ? 0.0 : last_sgn;
      P.status[gw] = singular;
    }
  }
}

template <typename T>
bool launch_sweep_reg(const Pools& P, const int32_t* wlist, int n_groups, int ne_max, int max_ns,
                      int max_M, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
                      const uint64_t* trace_base, const uint64_t* target, int32_t* needs_refresh,
                      int R, int kref, hipStream_t s) {
  constexpr int WPB = 4;
  if (n_groups <= 0 || cap <= 0) return true;
  const size_t sh = sweep_reg_lds_bytes(ne_max, max_ns, max_M, sizeof(T), WPB);
#define MVMC_REG_V(NEM, TR, RB)                                                                  \
  do {                                                                                           \
    if (sh > 65536)                                                                              \
      (void)hipFuncSetAttribute((const void*)&k_sweep_reg<T, NEM, WPB, TR, RB>,                  \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);            \
    hipLaunchKernelGGL((k_sweep_reg<T, NEM, WPB, TR, RB>), dim3(n_groups), dim3(64 * WPB), sh,   \
                       s, P, wlist, cap, seed, trace, trace_cap, trace_base, target,             \
                       needs_refresh, R, kref);                                                  \
    return true;                                                                                 \
  } while (0)
#define MVMC_REG(NEM)                                                                            \
  do {                                                                                           \
    if (trace) {                                                                                 \
      if (max_M > 0) MVMC_REG_V(NEM, true, true);                                                \
      MVMC_REG_V(NEM, true, false);                                                              \
    }                                                                                            \
    if (max_M > 0) MVMC_REG_V(NEM, false, true);                                                 \
    MVMC_REG_V(NEM, false, false);                                                               \
  } while (0)
  if (ne_max == 32) MVMC_REG(32);
  if (ne_max == 64) MVMC_REG(64);
#undef MVMC_REG_V
#undef MVMC_REG
  return false;
}

int sweep_reg_class(int ne, size_t tsize) {
  (void)tsize;
  if (ne <= 32) return 32;
  if (ne <= 64) return 64;
  return 0;
}

template bool launch_sweep_reg<double>(const Pools&, const int32_t*, int, int, int, int, int,
                                       uint64_t, TraceRec*, int64_t, const uint64_t*,
                                       const uint64_t*, int32_t*, int, int, hipStream_t);
template bool launch_sweep_reg<float>(const Pools&, const int32_t*, int, int, int, int, int,
                                      uint64_t, TraceRec*, int64_t, const uint64_t*,
                                      const uint64_t*, int32_t*, int, int, hipStream_t);

}  // namespace mvmc
