// Metropolis sweep kernel: one workgroup per walker, the walker's inverse
// Y = X^-1 resident in LDS for the whole launch (or in HBM when it does not
// fit), n_prop proposals per launch.
//
// Per proposal (hopping update, section 3.1.2 / Fig. 5a; ratio from the
// fast-update technique of section 3.1.2):
//   draw (r0..r3) = Philox(counter = (n, walker, 0));  a = (r0 N_e) >> 32;
//   target = empty_sigma[(r1 (Ns - N_sigma)) >> 32];  u = uniform53(r2, r3);
//   x'_b = A[I'][I_b] (b != a), x'_a = 0;
//   r_Pf = sum_b x'_b Y_ba = -sum_b Y_ab x'_b     (Pfaffian is affine in row a)
//   Gutzwiller:  g_k n_{k,~s} - g_i n_{i,~s};  Jastrow: h_k - h_i - v_ik
//   RBM: 2(a_I' - a_I) + sum_h [log 2cosh(theta_h + dtheta_h) - log 2cosh theta_h],
//        dtheta_h = 2 (W_hI' - W_hI)
//   R = r_Pf exp(sum of the correlator terms);  accept iff u < R^2.
// On acceptance the inverse gets the rank-2 update
//   p = Y e_a = -Y[a,:]^T,  q = Y x'_a + e_a,  Y <- Y + (p q^T - q p^T) / r_Pf
// (matrix-determinant lemma and Woodbury identity for X' = X + e_a u^T - u e_a^T),
// and pos, the empty list, the Jastrow field and the RBM angles follow.
#include "launch.h"

namespace mvmc {

namespace {
struct SweepLds {
  size_t Y, vec, qpart, h, th, red, ints, total;
};
__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline SweepLds sweep_layout(int ne, int ns, int M, bool lds, size_t ts,
                                                 int nw) {
  SweepLds L;
  L.Y = lds ? al16((size_t)ne * ne * ts) : 0;
  L.vec = al16(3 * (size_t)ne * ts);
  L.qpart = al16((size_t)nw * ne * ts);
  L.h = al16((size_t)ns * sizeof(double));
  L.th = al16((size_t)M * ts);
  L.red = al16(2 * (size_t)(nw > 8 ? nw : 8) * sizeof(double));
  L.ints = al16((size_t)(ne + 4 * ns) * sizeof(int32_t));
  L.total = L.Y + L.vec + L.qpart + L.h + L.th + L.red + L.ints;
  return L;
}

template <typename T> __device__ __forceinline__ const T* skew_table(const Pools& P, int64_t off);
template <> __device__ __forceinline__ const double* skew_table<double>(const Pools& P, int64_t off) {
  return P.A64 + off;
}
template <> __device__ __forceinline__ const float* skew_table<float>(const Pools& P, int64_t off) {
  return P.A32 + off;
}
template <typename T> __device__ __forceinline__ const T* rbm_pool(const Pools& P);
template <> __device__ __forceinline__ const double* rbm_pool<double>(const Pools& P) { return P.rbm64; }
template <> __device__ __forceinline__ const float* rbm_pool<float>(const Pools& P) { return P.rbm32; }
}  // namespace

size_t sweep_lds_bytes(int ne, int ns, int M, bool lds, size_t tsize, int nthreads) {
  return sweep_layout(ne, ns, M, lds, tsize, nthreads / 64).total;
}

// Each walker runs proposals up to its target counter, at most `cap` per
// launch and never past a multiple of refresh_every (R > 0) of its proposal
// counter, or of its applied-update counter when the pools say so: a walker
// that reaches such a multiple raises its refresh flag.
template <typename T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_sweep(Pools P, const int32_t* __restrict__ wlist,
                                              int cap, uint64_t seed, TraceRec* trace,
                                              int64_t trace_cap,
                                              const uint64_t* __restrict__ trace_base,
                                              const uint64_t* __restrict__ target,
                                              int32_t* __restrict__ needs_refresh, int R) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  const int32_t guard0 = P.guard[gw];
  if (guard0 == kGuardFailed) return;
  const uint64_t n0 = P.cnt[gw];
  const uint64_t tg = target[gw];
  uint64_t todo = tg > n0 ? tg - n0 : 0;
  if (todo > (uint64_t)cap) todo = (uint64_t)cap;
  const bool by_upd = P.refresh_upd != 0;
  if (R > 0 && !by_upd) {
    const uint64_t left = (uint64_t)R - n0 % (uint64_t)R;
    if (todo > left) todo = left;
  }
  if (todo == 0) return;
  const int n_prop = (int)todo;
  const uint64_t u0 = P.upd[gw];
  const uint64_t R_upd = by_upd && R > 0 ? (uint64_t)R : 0;   // R is the ratio inside the loop
  bool due = false;   // the applied update that completes a multiple of R was made
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, M = I.M, nup = I.nup;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  const SweepLds L = sweep_layout(ne, ns, M, LDS, sizeof(T), NW);
  unsigned char* q = smem;
  T* Yg = (T*)P.Y + I.Y_off + lw * ne * ne;
  T* Y = LDS ? (T*)q : Yg;
  q += L.Y;
  T* xn = (T*)q;
  T* pv = xn + ne;
  T* qv = pv + ne;
  q += L.vec;
  T* qpart = (T*)q;
  q += L.qpart;
  double* hs = (double*)q;
  q += L.h;
  T* ths = (T*)q;
  q += L.th;
  double* red = (double*)q;
  q += L.red;
  int32_t* pos_s = (int32_t*)q;
  int32_t* eidx = pos_s + ne;     // 2ns: electron at spin-orbital, -1 empty
  int32_t* emp = eidx + n2;       // 2ns: empty lists [sigma][ns]

  int32_t* posg = P.pos + I.pos_off + lw * ne;
  int32_t* empg = P.empty + I.empty_off + lw * n2;
  double* hg = P.h + I.h_off + lw * ns;
  double* thg = P.theta + I.theta_off + lw * M;

  if (LDS)
    for (int e = tid; e < ne * ne; e += NT) Y[e] = Yg[e];
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

  const T* A = skew_table<T>(P, I.A_off);
  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const T* ra = rbm_pool<T>(P) + I.rbm_a_off;
  const T* rW = rbm_pool<T>(P) + I.rbm_W_off;
  const uint64_t tb = trace ? trace_base[gw] : 0;
  int64_t acc = 0;
  // A ratio that is not finite stops the walker at that proposal and asks
  // for a double refresh before it is tried again; not finite again right
  // after that refresh, the walker stops for good (kGuardFailed).
  int n_done = n_prop;
  int32_t guard1 = guard0;

  for (int it = 0; it < n_prop; ++it) {
    const uint64_t n = n0 + (uint64_t)it;
    const uint4 r = draw(seed, n, (uint32_t)gw, 0u);
    const int a = scaled(r.x, ne);
    const int sigma = a >= nup ? 1 : 0;
    const int nemp = ns - (sigma ? I.ndn : nup);
    if (nemp == 0) {
      if (trace && tid == 0 && n - tb < (uint64_t)trace_cap) {
        TraceRec rec;
        rec.b = -1; rec.pad = 0;
        rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = -1; rec.accepted = 0;
        rec.ratio = 0.0;
        trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
      }
      continue;
    }
    const int k = scaled(r.y, nemp);
    const int site_new = emp[sigma * ns + k];
    const int Inew = site_new + sigma * ns;
    const int Iold = pos_s[a];
    const int site_old = Iold - sigma * ns;

    // Pfaffian ratio: dot of the new row a of X with row a of Y.  With the
    // anti-parallel pair amplitude (Eq. AP-Pf) the new row of X vanishes on
    // the electrons of a's own spin, and so do the same-spin blocks of Y
    // ([[0, -M^-T], [M^-1, 0]]): only the opposite-spin electrons enter.
    const int o0 = sigma ? 0 : nup, o1 = sigma ? nup : ne;   // opposite spin
    const int s0 = sigma ? nup : 0, s1 = sigma ? ne : nup;   // a's spin
    const T* Arow = A + (int64_t)Inew * n2;
    const T* Ya = Y + a * ne;
    T accp = T(0);
    for (int b = o0 + tid; b < o1; b += NT) {
      const T xb = Arow[pos_s[b]];
      xn[b] = xb;
      accp += xb * Ya[b];
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
    const double r_pf = -sp;
    const int opp = (1 - sigma) * ns;
    double logc = G[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  G[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                  hs[site_old] - V[(int64_t)site_old * ns + site_new];
    if (M) logc += 2.0 * ((double)ra[Inew] - (double)ra[Iold]) + sr;
    const double R = r_pf * exp(logc);
    if (!isfinite(R)) {   // uniform: every thread holds the same sums
      guard1 = guard1 == kGuardPending ? kGuardFailed : kGuardPending;
      n_done = it;
      break;
    }
    guard1 = kGuardClear;
    const double u = uniform53(r.z, r.w);
    const bool accept = u < R * R;
    if (trace && tid == 0 && n - tb < (uint64_t)trace_cap) {
      TraceRec rec;
      rec.b = -1; rec.pad = 0;
      rec.n = (int64_t)n; rec.walker = gw; rec.a = a; rec.i_new = Inew;
      rec.accepted = accept ? 1 : 0; rec.ratio = R;
      trace[(int64_t)gw * trace_cap + (int64_t)(n - tb)] = rec;
    }
    if (!accept) continue;
    ++acc;
    __syncthreads();   // x' visible to every thread

    // p = -Y[a,:] lives on the opposite spin, q = -Y^T x' + e_a on a's spin
    // (x' is zero on a's spin and Y's same-spin blocks are zero), so only
    // the two opposite-spin blocks of Y are read and updated; the same-spin
    // blocks would receive exact zeros.
    for (int i = o0 + tid; i < o1; i += NT) pv[i] = -Ya[i];
    {
      const int no = o1 - o0;
      const int j0 = o0 + (wid * no) / NW, j1 = o0 + ((wid + 1) * no) / NW;
      for (int i = s0 + lane; i < s1; i += 64) {
        T sq = T(0);
        for (int j = j0; j < j1; ++j) sq += Y[j * ne + i] * xn[j];
        qpart[wid * ne + i] = sq;
      }
    }
    __syncthreads();
    for (int i = s0 + tid; i < s1; i += NT) {
      T sq = T(0);
#pragma unroll
      for (int w = 0; w < NW; ++w) sq += qpart[w * ne + i];
      qv[i] = (i == a ? T(1) : T(0)) - sq;
    }
    __syncthreads();
    const T ir = T(1.0 / r_pf);
    // rows of a's spin: Y[r][c] -= q_r p_c / r_Pf over the opposite-spin columns;
    // rows of the opposite spin: Y[r][c] += p_r q_c / r_Pf over a's spin
    for (int rr = wid; rr < ne; rr += NW) {
      T* Yr = Y + rr * ne;
      if (rr >= s0 && rr < s1) {
        const T qr = qv[rr] * ir;
        for (int c = o0 + lane; c < o1; c += 64) Yr[c] -= qr * pv[c];
      } else {
        const T pr = pv[rr] * ir;
        for (int c = s0 + lane; c < s1; c += 64) Yr[c] += pr * qv[c];
      }
    }
    // V is symmetric: row site_new read across the threads is coalesced
    for (int l = tid; l < ns; l += NT) hs[l] += V[(int64_t)site_new * ns + l] - V[(int64_t)site_old * ns + l];
    for (int hh = tid; hh < M; hh += NT)
      ths[hh] += T(2) * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
    if (tid == 0) {
      pos_s[a] = Inew;
      eidx[Iold] = -1;
      eidx[Inew] = a;
      emp[sigma * ns + k] = site_old;
    }
    __syncthreads();
    if (R_upd && (u0 + (uint64_t)acc) % R_upd == 0) {   // uniform
      due = true;
      n_done = it + 1;
      break;
    }
  }

  __syncthreads();
  if (LDS)
    for (int e = tid; e < ne * ne; e += NT) Yg[e] = Y[e];
  for (int b = tid; b < ne; b += NT) posg[b] = pos_s[b];
  for (int v = tid; v < n2; v += NT) empg[v] = emp[v];
  for (int l = tid; l < ns; l += NT) hg[l] = hs[l];
  for (int hh = tid; hh < M; hh += NT) thg[hh] = (double)ths[hh];
  if (tid == 0) {
    const uint64_t n1 = n0 + (uint64_t)n_done;
    P.cnt[gw] = n1;
    P.upd[gw] = u0 + (uint64_t)acc;
    P.accepted[gw] += acc;
    if (guard1 != guard0) P.guard[gw] = guard1;
    if ((R > 0 && (by_upd ? due : n1 % (uint64_t)R == 0)) || guard1 == kGuardPending)
      needs_refresh[gw] = 1;
  }
}

template <typename T>
void launch_sweep(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                  int max_ne, int max_ns, int max_M, bool lds, int nthreads, TraceRec* trace,
                  int64_t trace_cap, const uint64_t* trace_base, const uint64_t* target,
                  int32_t* needs_refresh, int R, hipStream_t s) {
  if (n <= 0 || cap <= 0) return;
  const int nw = nthreads / 64;
  const size_t sh = sweep_layout(max_ne, max_ns, max_M, lds, sizeof(T), nw).total;
#define MVMC_SWEEP_LAUNCH(LDSV, NTV)                                                           \
  do {                                                                                         \
    if (sh > 65536)                                                                            \
      (void)hipFuncSetAttribute((const void*)&k_sweep<T, LDSV, NTV>,                                \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);                \
    hipLaunchKernelGGL((k_sweep<T, LDSV, NTV>), dim3(n), dim3(NTV), sh, s, P, wlist, cap, seed, \
                       trace, trace_cap, trace_base, target, needs_refresh, R);                \
  } while (0)
  if (lds) {
    if (nthreads == 64) MVMC_SWEEP_LAUNCH(true, 64);
    else if (nthreads == 128) MVMC_SWEEP_LAUNCH(true, 128);
    else MVMC_SWEEP_LAUNCH(true, 256);
  } else {
    if (nthreads == 64) MVMC_SWEEP_LAUNCH(false, 64);
    else if (nthreads == 128) MVMC_SWEEP_LAUNCH(false, 128);
    else MVMC_SWEEP_LAUNCH(false, 256);
  }
#undef MVMC_SWEEP_LAUNCH
}

template void launch_sweep<double>(const Pools&, const int32_t*, int, int, uint64_t, int, int, int,
                                   bool, int, TraceRec*, int64_t, const uint64_t*,
                                   const uint64_t*, int32_t*, int, hipStream_t);
template void launch_sweep<float>(const Pools&, const int32_t*, int, int, uint64_t, int, int, int,
                                  bool, int, TraceRec*, int64_t, const uint64_t*,
                                  const uint64_t*, int32_t*, int, hipStream_t);

}  // namespace mvmc
