// Quantum-number projection of the pair-product part (section 3.2.2, Eqs.
// momP and pointP) on the anti-parallel block: refresh and sweep.
//
// psi(x) = P_G P_J [RBM] sum_p w_p Pf(X(q_p(x))): term p is the Pfaffian of
// the configuration whose electrons sit on the images q_p(i) of their sites
// (spin and electron order kept).  With the anti-parallel pair amplitude
// (Eq. AP-Pf) that Pfaffian is (-1)^{n(n-1)/2} det M_p with
//     M_p[a][b] = f(q_p(s_a), q_p(s_b))   (up electron a, down electron b),
// and a walker keeps every M_p^-1 (n x n, n = N_e/2) with l_p = log|det M_p|
// and its sign.  A hop of electron a changes row a (up) or column a (down) of
// every M_p, so the determinant lemma gives each term's ratio r_p from M_p^-1
// exactly as without projection, and the pair-product ratio is
//     R_Pf = sum_p c_p r_p / sum_p c_p,   c_p = w_p sgn_p exp(l_p - max l).
// On acceptance every M_p^-1 takes its rank-1 Sherman-Morrison update and
// l_p += log|r_p|, sgn_p *= sign(r_p).  The Gutzwiller, Jastrow and RBM
// factors do not depend on p and follow the unprojected sweep.
//
// Walker storage: block p of the walker's matrix space holds M_p^-1 with
// entry [b][a] (down b, up a) at p n^2 + b n + a; the pterm pool holds l_p
// then sgn_p; logpf / sgnpf hold log|sum_p w_p Pf_p| and its sign.
#include "common.h"
#include "launch.h"

namespace mvmc {

namespace {
constexpr int kProjThreads = 256;
constexpr int kProjWaves = kProjThreads / 64;
__host__ __device__ inline size_t pj16(size_t x) { return (x + 15) & ~(size_t)15; }

// ------------------------------------------------------------------ refresh
// LDS: tableau [n][n + 1] double, pivot row and column copies [n] each,
// reduction scratch, then ints: positions [N_e], occupations [2 N_s], pivot
// row of each column [n], used rows [n], two words.
__host__ __device__ inline size_t proj_refresh_lds(int ne, int ns) {
  const int n = ne / 2;
  return pj16(((size_t)n * (n + 1) + 2 * (size_t)n + 2 * kProjWaves) * sizeof(double)) +
         (size_t)(ne + 2 * ns + 2 * n + 2) * sizeof(int32_t);
}

// One workgroup per walker: every term's M_p by Gauss-Jordan exchange steps
// with partial pivoting in double (the elimination of ap_refresh.h, here
// with the tableau in LDS): step k takes the unused row p of largest
// |T[r][k]|, pi = T[p][k], and sets T[p][k] = 1/pi, T[p][c] = -T[p][c]/pi,
// T[r][k] = T[r][k]/pi, T[r][c] -= T[r][k] T[p][c]/pi.  Afterwards, with p_k
// the pivot row of column k, M^-1[k][p_j] = T[p_k][j] (first index a column of
// M, i.e. a down electron; second a row, an up electron) and
// det M = sgn(k -> p_k) prod pi_k.  Then the sum
// over terms, the Jastrow field and the RBM angles.  A term whose pivot falls
// to sing_tol times its largest entry (or to zero) marks the walker singular.
template <typename T>
__global__ __launch_bounds__(kProjThreads) void k_refresh_proj(Pools P,
                                                               const int32_t* __restrict__ wlist,
                                                               double sing_tol,
                                                               int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  if (gw < 0 || (flags && !flags[gw])) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, nh = I.nup, np = I.nproj;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ld = nh + 1;

  double* Tt = (double*)smem;
  double* prow = Tt + (size_t)nh * ld;
  double* pcol = prow + nh;
  double* red = pcol + nh;                          // 2 * kProjWaves
  int32_t* pos = (int32_t*)(smem + pj16(((size_t)nh * ld + 2 * (size_t)nh + 2 * kProjWaves) *
                                        sizeof(double)));
  int32_t* occ = pos + ne;
  int32_t* piv = occ + n2;
  int32_t* used = piv + nh;
  int32_t* word = used + nh;                        // [0] pivot row

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int b = tid; b < ne; b += kProjThreads) pos[b] = posg[b];
  for (int v = tid; v < n2; v += kProjThreads) occ[v] = 0;
  __syncthreads();
  for (int b = tid; b < ne; b += kProjThreads) occ[pos[b]] = 1;

  const double* A = P.A64 + I.A_off;
  const int32_t* qall = P.pmap + I.proj_off;
  const double* wts = P.projw + I.projw_off;
  double* lterm = P.pterm + I.pterm_off + lw * 2 * np;
  double* sterm = lterm + np;
  T* Yw = (T*)P.Y + I.Y_off + lw * I.Y_ld;
  bool any_singular = false;
  double minpiv_all = INFINITY;
  for (int p = 0; p < np; ++p) {
    const int32_t* q = qall + (size_t)p * ns;
    __syncthreads();   // previous term's tableau fully read
    double amax = 0.0;
    for (int e = tid; e < nh * nh; e += kProjThreads) {
      const int a = e / nh, b = e - (e / nh) * nh;
      const double v = A[(int64_t)q[pos[a]] * n2 + ns + q[pos[nh + b] - ns]];
      Tt[a * ld + b] = v;
      amax = fmax(amax, fabs(v));
    }
    for (int r = tid; r < nh; r += kProjThreads) used[r] = 0;
    // largest |entry| over the workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) red[wid] = amax;
    __syncthreads();
    amax = 0.0;
#pragma unroll
    for (int w = 0; w < kProjWaves; ++w) amax = fmax(amax, red[w]);
    double logabs = 0.0, sgn = 1.0, minpiv = INFINITY;
    bool singular = false;
    for (int k = 0; k < nh; ++k) {
      if (wid == 0) {
        // unused row of largest |T[r][k]|, lowest row on ties
        double best = -1.0;
        int bi = nh;
        for (int r = lane; r < nh; r += 64)
          if (!used[r]) {
            const double v = fabs(Tt[r * ld + k]);
            if (v > best) {
              best = v;
              bi = r;
            }
          }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (lane == 0) {
          word[0] = bi;
          used[bi] = 1;
          piv[k] = bi;
        }
      }
      __syncthreads();
      const int pr = word[0];
      const double pi = Tt[pr * ld + k];
      if (!(fabs(pi) > sing_tol * amax) || pi == 0.0) {   // uniform across the workgroup
        singular = true;
        break;
      }
      logabs += log(fabs(pi));
      if (pi < 0.0) sgn = -sgn;
      minpiv = fmin(minpiv, fabs(pi));
      for (int c = tid; c < nh; c += kProjThreads) {
        prow[c] = Tt[pr * ld + c];
        pcol[c] = Tt[c * ld + k];
      }
      __syncthreads();
      const double ipi = 1.0 / pi;
      for (int e = tid; e < nh * nh; e += kProjThreads) {
        const int r = e / nh, c = e - (e / nh) * nh;
        double v;
        if (r == pr) v = c == k ? ipi : -prow[c] * ipi;
        else if (c == k) v = pcol[r] * ipi;
        else v = Tt[r * ld + c] - pcol[r] * prow[c] * ipi;
        Tt[r * ld + c] = v;
      }
      __syncthreads();
    }
    if (singular) {
      any_singular = true;
      if (tid == 0) {
        lterm[p] = -INFINITY;
        sterm[p] = 0.0;
      }
      continue;
    }
    // M_p^-1[k][p_j] = T[p_k][j], stored at k n + p_j
    T* Yp = Yw + (int64_t)p * nh * nh;
    for (int e = tid; e < nh * nh; e += kProjThreads) {
      const int k = e / nh, j = e - (e / nh) * nh;
      Yp[k * nh + piv[j]] = (T)Tt[piv[k] * ld + j];
    }
    if (tid == 0) {
      // sign of the permutation k -> p_k by its cycles, then (-1)^{n(n-1)/2}
      for (int r = 0; r < nh; ++r) used[r] = 0;
      int parity = 0;
      for (int k = 0; k < nh; ++k) {
        if (used[k]) continue;
        int len = 0;
        for (int j = k; !used[j]; j = piv[j]) {
          used[j] = 1;
          ++len;
        }
        parity += len - 1;
      }
      if (parity & 1) sgn = -sgn;
      if (((nh * (nh - 1)) / 2) & 1) sgn = -sgn;
      lterm[p] = logabs;
      sterm[p] = sgn;
    }
    minpiv_all = fmin(minpiv_all, minpiv / (amax > 0.0 ? amax : 1.0));
  }
  __syncthreads();
  if (tid == 0) {
    double lmax = -INFINITY;
    for (int p = 0; p < np; ++p)
      if (sterm[p] != 0.0) lmax = fmax(lmax, lterm[p]);
    double tot = 0.0;
    for (int p = 0; p < np; ++p)
      if (sterm[p] != 0.0) tot += wts[p] * sterm[p] * exp(lterm[p] - lmax);
    const bool bad = any_singular || !(tot != 0.0) || !isfinite(tot);
    if (flags) flags[gw] = 0;
    P.logpf[gw] = bad ? -INFINITY : lmax + log(fabs(tot));
    P.sgnpf[gw] = bad ? 0.0 : (tot > 0.0 ? 1.0 : -1.0);
    P.minpiv[gw] = any_singular ? 0.0 : minpiv_all;
    P.status[gw] = bad ? 1 : 0;
  }

  // Jastrow field h_l = sum_m v_lm (n_m - 1) and RBM angles theta = b + W sigma
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  for (int l = tid; l < ns; l += kProjThreads) {
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
    for (int hh = tid; hh < I.M; hh += kProjThreads) {
      double s = bb[hh];
      for (int v = 0; v < n2; ++v) s += WT[(int64_t)v * I.M + hh] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

// -------------------------------------------------------------------- sweep
struct ProjLds {
  size_t Mi, vec, h, th, red, terms, ints, total;
  int ld;
};
// Row stride n + 1 for even n (odd strides spread the strided column reads
// over the LDS banks).
__host__ __device__ inline ProjLds proj_sweep_layout(int ne, int ns, int M, int np, size_t ts) {
  ProjLds L;
  const int n = ne / 2;
  L.ld = n + ((n & 1) ? 0 : 1);
  L.Mi = pj16((size_t)np * n * L.ld * ts);
  L.vec = pj16(3 * (size_t)np * n * ts);            // m'_p, column/row of M_p^-1, v_p or t_p
  L.h = pj16((size_t)ns * sizeof(double));
  L.th = pj16((size_t)M * ts);
  L.red = pj16(2 * 8 * sizeof(double));
  L.terms = pj16(5 * (size_t)np * sizeof(double));  // l_p, sgn_p, w_p, r_p (two buffers)
  L.ints = pj16((size_t)(ne + 4 * ns + np * ns) * sizeof(int32_t));
  L.total = L.Mi + L.vec + L.h + L.th + L.red + L.terms + L.ints;
  return L;
}

template <typename T> __device__ __forceinline__ const T* pj_table(const Pools& P, int64_t off);
template <> __device__ __forceinline__ const double* pj_table<double>(const Pools& P, int64_t off) {
  return P.A64 + off;
}
template <> __device__ __forceinline__ const float* pj_table<float>(const Pools& P, int64_t off) {
  return P.A32 + off;
}
template <typename T> __device__ __forceinline__ const T* pj_rbm(const Pools& P);
template <> __device__ __forceinline__ const double* pj_rbm<double>(const Pools& P) { return P.rbm64; }
template <> __device__ __forceinline__ const float* pj_rbm<float>(const Pools& P) { return P.rbm32; }

// One workgroup per walker; wavefront w carries terms w, w + 4, ...  The
// proposal draw and stopping rule are those of the unprojected sweeps (the
// same Philox stream, refresh at every multiple of R proposals or applied
// updates, non-finite guard).
template <typename T>
__global__ __launch_bounds__(kProjThreads) void k_sweep_proj(
    Pools P, const int32_t* __restrict__ wlist, int cap, uint64_t seed, TraceRec* trace,
    int64_t trace_cap, const uint64_t* __restrict__ trace_base, const uint64_t* __restrict__ target,
    int32_t* __restrict__ needs_refresh, int R) {
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
  const uint64_t u0 = P.upd[gw];
  bool due = false;   // the applied update that completes a multiple of R was made
  const int n_prop = (int)todo;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, M = I.M, n = I.nup, np = I.nproj;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  const ProjLds L = proj_sweep_layout(ne, ns, M, np, sizeof(T));
  const int ld = L.ld;
  unsigned char* q = smem;
  T* Mi = (T*)q;                  // block p: M_p^-1[i][j] at p n ld + i ld + j
  q += L.Mi;
  T* mv = (T*)q;                  // [p][n] new row (up) or column (down) of M_p
  T* cr = mv + (size_t)np * n;    // [p][n] column a (up) or row a (down) of M_p^-1
  T* vt = cr + (size_t)np * n;    // [p][n] v_p (up) or t_p (down)
  q += L.vec;
  double* hs = (double*)q;
  q += L.h;
  T* ths = (T*)q;
  q += L.th;
  double* red = (double*)q;
  q += L.red;
  double* lg = (double*)q;        // l_p
  double* sg = lg + np;           // sgn_p
  double* wt = sg + np;           // w_p
  // r_p of the current proposal, alternating between two buffers: a
  // rejected proposal ends without a barrier, so the next one must not
  // overwrite values other wavefronts may still be reading
  double* rp2 = wt + np;
  q += L.terms;
  int32_t* pos_s = (int32_t*)q;
  int32_t* eidx = pos_s + ne;     // 2ns: electron at spin-orbital, -1 empty
  int32_t* emp = eidx + n2;       // 2ns: empty lists [sigma][ns]
  int32_t* qm = emp + n2;         // [p][ns] site maps

  T* Yw = (T*)P.Y + I.Y_off + lw * I.Y_ld;
  int32_t* posg = P.pos + I.pos_off + lw * ne;
  int32_t* empg = P.empty + I.empty_off + lw * n2;
  double* hg = P.h + I.h_off + lw * ns;
  double* thg = P.theta + I.theta_off + lw * M;
  double* ltg = P.pterm + I.pterm_off + lw * 2 * np;

  for (int e = tid; e < np * n * n; e += kProjThreads) {
    const int p = e / (n * n), r = e - p * n * n, i = r / n, j = r - (r / n) * n;
    Mi[(size_t)p * n * ld + i * ld + j] = Yw[e];
  }
  for (int v = tid; v < n2; v += kProjThreads) {
    eidx[v] = -1;
    emp[v] = empg[v];
  }
  for (int e = tid; e < np * ns; e += kProjThreads) qm[e] = P.pmap[I.proj_off + e];
  for (int p = tid; p < np; p += kProjThreads) {
    lg[p] = ltg[p];
    sg[p] = ltg[np + p];
    wt[p] = P.projw[I.projw_off + p];
  }
  for (int l = tid; l < ns; l += kProjThreads) hs[l] = hg[l];
  for (int hh = tid; hh < M; hh += kProjThreads) ths[hh] = (T)thg[hh];
  __syncthreads();
  for (int b = tid; b < ne; b += kProjThreads) {
    const int v = posg[b];
    pos_s[b] = v;
    eidx[v] = b;
  }
  __syncthreads();

  const T* A = pj_table<T>(P, I.A_off);
  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const T* ra = pj_rbm<T>(P) + I.rbm_a_off;
  const T* rW = pj_rbm<T>(P) + I.rbm_W_off;
  const uint64_t tb = trace ? trace_base[gw] : 0;
  int64_t acc = 0;
  int32_t guard1 = guard0;

  int it = 0;
  while (it < n_prop) {
    const uint64_t nn = n0 + (uint64_t)it;
    const uint4 r = draw(seed, nn, (uint32_t)gw, 0u);
    double* rp = rp2 + (it & 1) * np;
    bool nonfinite = false;
    do {   // one proposal; `continue` ends it
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
      const int ai = a - sigma * n;   // row (up) or column (down) of every M_p

      // r_p and the vectors its update needs, one wavefront per term
      for (int p = wid; p < np; p += kProjWaves) {
        const int32_t* qp = qm + p * ns;
        const T* Mp = Mi + (size_t)p * n * ld;
        T* mvp = mv + p * n;
        T* crp = cr + p * n;
        T s = T(0);
        if (sigma == 0) {
          const T* Arow = A + (int64_t)qp[site_new] * n2 + ns;   // f(q(s'), .)
          for (int b = lane; b < n; b += 64) {
            const T x = Arow[qp[pos_s[n + b] - ns]];
            const T c = Mp[b * ld + ai];
            mvp[b] = x;
            crp[b] = c;
            s += x * c;
          }
        } else {
          // f(q(s_i), q(s')) = -A[(q(s'), dn)][(q(s_i), up)]: a row of the table
          const T* Acol = A + (int64_t)(ns + qp[site_new]) * n2;
          for (int i = lane; i < n; i += 64) {
            const T x = -Acol[qp[pos_s[i]]];
            const T c = Mp[ai * ld + i];
            mvp[i] = x;
            crp[i] = c;
            s += c * x;
          }
        }
        s = wave_sum(s);
        if (lane == 0) rp[p] = (double)s;
      }
      double accr = 0.0;
      if (M) {
        for (int hh = tid; hh < M; hh += kProjThreads) {
          const T d = T(2) * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
          const T th = ths[hh];
          accr += (double)(log2cosh(th + d) - log2cosh(th));
        }
      }
      accr = block_sum(accr, red);
      __syncthreads();   // r_p and the per-term vectors for every thread
      double lmax = -INFINITY;
      for (int p = 0; p < np; ++p)
        if (sg[p] != 0.0) lmax = fmax(lmax, lg[p]);
      double num = 0.0, den = 0.0;
      bool zero_term = false;
      for (int p = 0; p < np; ++p) {
        if (sg[p] == 0.0) continue;   // no inverse to update (kept only for robustness)
        const double c = wt[p] * sg[p] * exp(lg[p] - lmax);
        num += c * rp[p];
        den += c;
        zero_term = zero_term || !(rp[p] != 0.0);
      }
      const double r_pf = num / den;
      const int opp = (1 - sigma) * ns;
      double logc = G[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                    G[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                    hs[site_old] - V[(int64_t)site_old * ns + site_new];
      if (M) logc += 2.0 * ((double)ra[Inew] - (double)ra[Iold]) + accr;
      const double Rt = r_pf * exp(logc);
      if (!isfinite(Rt)) {   // uniform: every thread holds the same sums
        nonfinite = true;
        continue;
      }
      const double u = uniform53(r.z, r.w);
      const bool accept = u < Rt * Rt;
      // an accepted move that makes one M_p singular cannot be followed by
      // its rank-1 update: handled like a non-finite ratio
      if (accept && zero_term) {
        nonfinite = true;
        continue;
      }
      guard1 = kGuardClear;
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
      // v_p = m'_p^T M_p^-1 - e_a (up) or t_p = M_p^-1 m'_p - e_a (down)
      for (int p = wid; p < np; p += kProjWaves) {
        const T* Mp = Mi + (size_t)p * n * ld;
        const T* mvp = mv + p * n;
        T* vtp = vt + p * n;
        for (int o = lane; o < n; o += 64) {
          T s = T(0);
          if (sigma == 0)
            for (int b = 0; b < n; ++b) s += mvp[b] * Mp[b * ld + o];
          else
            for (int j = 0; j < n; ++j) s += Mp[o * ld + j] * mvp[j];
          vtp[o] = s - (o == ai ? T(1) : T(0));
        }
      }
      __syncthreads();
      // up:   M_p^-1[i][j] -= cr[i] v[j] / r_p;   down: M_p^-1[i][j] -= t[i] cr[j] / r_p
      for (int p = wid; p < np; p += kProjWaves) {
        T* Mp = Mi + (size_t)p * n * ld;
        const T* crp = cr + p * n;
        const T* vtp = vt + p * n;
        const T ir = T(1.0 / rp[p]);
        for (int e = lane; e < n * n; e += 64) {
          const int i = e / n, j = e - (e / n) * n;
          const T lft = sigma == 0 ? crp[i] : vtp[i];
          const T rgt = sigma == 0 ? vtp[j] : crp[j];
          Mp[i * ld + j] -= (lft * ir) * rgt;
        }
        if (lane == 0) {
          lg[p] += log(fabs(rp[p]));
          if (rp[p] < 0.0) sg[p] = -sg[p];
        }
      }
      for (int l = tid; l < ns; l += kProjThreads)
        hs[l] += V[(int64_t)site_new * ns + l] - V[(int64_t)site_old * ns + l];
      for (int hh = tid; hh < M; hh += kProjThreads)
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
  for (int e = tid; e < np * n * n; e += kProjThreads) {
    const int p = e / (n * n), r = e - p * n * n, i = r / n, j = r - (r / n) * n;
    Yw[e] = Mi[(size_t)p * n * ld + i * ld + j];
  }
  for (int b = tid; b < ne; b += kProjThreads) posg[b] = pos_s[b];
  for (int v = tid; v < n2; v += kProjThreads) empg[v] = emp[v];
  for (int l = tid; l < ns; l += kProjThreads) hg[l] = hs[l];
  for (int hh = tid; hh < M; hh += kProjThreads) thg[hh] = (double)ths[hh];
  for (int p = tid; p < np; p += kProjThreads) {
    ltg[p] = lg[p];
    ltg[np + p] = sg[p];
  }
  const uint64_t n1 = n0 + (uint64_t)it;
  const bool stop = (R > 0 && (by_upd ? due : n1 % (uint64_t)R == 0)) ||
                    guard1 == kGuardPending;
  if (tid == 0) {
    double lmax = -INFINITY;
    for (int p = 0; p < np; ++p)
      if (sg[p] != 0.0) lmax = fmax(lmax, lg[p]);
    double tot = 0.0;
    for (int p = 0; p < np; ++p)
      if (sg[p] != 0.0) tot += wt[p] * sg[p] * exp(lg[p] - lmax);
    P.logpf[gw] = lmax + log(fabs(tot));
    P.sgnpf[gw] = tot > 0.0 ? 1.0 : (tot < 0.0 ? -1.0 : 0.0);
    P.cnt[gw] = n1;
    P.upd[gw] = u0 + (uint64_t)acc;
    P.accepted[gw] += acc;
    if (guard1 != guard0) P.guard[gw] = guard1;
    if (stop && needs_refresh) needs_refresh[gw] = 1;
  }
}
}  // namespace

size_t refresh_proj_lds_bytes(int ne, int ns) { return proj_refresh_lds(ne, ns); }

size_t sweep_proj_lds_bytes(int ne, int ns, int M, int nproj, size_t tsize) {
  return proj_sweep_layout(ne, ns, M, nproj, tsize).total;
}

template <typename T>
void launch_refresh_proj(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                         double sing_tol, int32_t* flags, hipStream_t s) {
  if (n <= 0) return;
  const size_t sh = proj_refresh_lds(max_ne, max_ns);
  if (sh > 65536)
    (void)hipFuncSetAttribute((const void*)&k_refresh_proj<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((k_refresh_proj<T>), dim3(n), dim3(kProjThreads), sh, s, P, wlist, sing_tol,
                     flags);
}

template <typename T>
void launch_sweep_proj(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                       size_t lds_bytes, TraceRec* trace, int64_t trace_cap,
                       const uint64_t* trace_base, const uint64_t* target, int32_t* needs_refresh,
                       int R, hipStream_t s) {
  if (n <= 0) return;
  if (lds_bytes > 65536)
    (void)hipFuncSetAttribute((const void*)&k_sweep_proj<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  hipLaunchKernelGGL((k_sweep_proj<T>), dim3(n), dim3(kProjThreads), lds_bytes, s, P, wlist, cap,
                     seed, trace, trace_cap, trace_base, target, needs_refresh, R);
}

template void launch_refresh_proj<double>(const Pools&, const int32_t*, int, int, int, double,
                                          int32_t*, hipStream_t);
template void launch_refresh_proj<float>(const Pools&, const int32_t*, int, int, int, double,
                                         int32_t*, hipStream_t);
template void launch_sweep_proj<double>(const Pools&, const int32_t*, int, int, uint64_t, size_t,
                                        TraceRec*, int64_t, const uint64_t*, const uint64_t*,
                                        int32_t*, int, hipStream_t);
template void launch_sweep_proj<float>(const Pools&, const int32_t*, int, int, uint64_t, size_t,
                                       TraceRec*, int64_t, const uint64_t*, const uint64_t*,
                                       int32_t*, int, hipStream_t);

}  // namespace mvmc
