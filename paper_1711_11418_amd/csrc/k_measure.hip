// Local energy and log-derivatives for one sample slot, one workgroup per walker.
//
// E_loc(x) = sum_x' <x|H|x'> psi(x')/psi(x)  (section 3.1.1, Eq. MC) for
// H = H_T + H_U (section 2.3): the diagonal sum_i U_i n_iup n_idn plus, for
// every electron a and every neighbour j of its site with (j, sigma_a) empty,
// -t * R(a -> j), R read from the current inverse exactly as in the sweep
// (the moved electron keeps its row, which carries the fermion sign).
//
// O_k = d ln<x|psi>/d alpha_k (section 3.3.1):
//   f slot k : -sum over members (i, j) of Y[a(i,up)][b(j,dn)]  (Eq. DiffPf,
//              appendix C: dPf/dF_AB = -Pf (X^-1)_AB)
//   g slot k : sum over member sites of n_iup n_idn
//   v slot k : sum over member pairs i < j of (n_i - 1)(n_j - 1)
//   RBM      : sigma_v, tanh theta_h, tanh theta_h sigma_v
// Rows are written in the parameter-vector order; padding columns are zeroed.
#include "launch.h"

namespace mvmc {

namespace {
constexpr int kMeasureThreads = 256;
// Sum over the members of each parameter slot: a group of G lanes per slot,
// lanes stride over the members, fixed-order shuffle reduction inside the
// group (deterministic).  G is picked from the mean members per slot.
template <int G, typename T, typename F>
__device__ __forceinline__ void slot_sums(int nslot, const int32_t* __restrict__ ptr,
                                          const int32_t* __restrict__ mem, F val,
                                          T* __restrict__ out) {
  const int lane_in = threadIdx.x & (G - 1);
  const int grp = threadIdx.x / G, ngrp = blockDim.x / G;
  for (int k = grp; k < nslot; k += ngrp) {
    double s = 0.0;
#pragma unroll 8
    for (int m = ptr[k] + lane_in; m < ptr[k + 1]; m += G) s += val(mem[m]);
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane_in == 0) out[k] = (T)s;
  }
}

template <typename T, typename F>
__device__ __forceinline__ void slot_sums_any(int nslot, int nmem, const int32_t* ptr,
                                              const int32_t* mem, F val, T* out) {
  const int avg = nslot > 0 ? (nmem + nslot - 1) / nslot : 0;
  // one lane per slot while a slot has few members (independent loads, no
  // cross-lane reduction); lane groups for slots with many members
  if (avg <= 32) slot_sums<1>(nslot, ptr, mem, val, out);
  else if (avg <= 256) slot_sums<16>(nslot, ptr, mem, val, out);
  else slot_sums<64>(nslot, ptr, mem, val, out);
}

template <typename T> __device__ __forceinline__ const T* table_of(const Pools& P, int64_t off);
template <> __device__ __forceinline__ const double* table_of<double>(const Pools& P, int64_t off) {
  return P.A64 + off;
}
template <> __device__ __forceinline__ const float* table_of<float>(const Pools& P, int64_t off) {
  return P.A32 + off;
}
}  // namespace

// LDS carve-up: [red 16 | hs ns | ths M] doubles, [Yh ne*(ne/2+1) | f ns*(ns+1)] T, ints.
// Yh keeps, for every electron a, only the entries of row a of Y on the
// electrons of the other spin (b >= n_up for an up electron, b < n_up for a
// down one): with the anti-parallel pair amplitude the new row a of X vanishes
// on the electrons of a's own spin, and the f log-derivatives pair an up with
// a down electron, so no other entry of Y enters the measurement.
__host__ __device__ inline size_t mal16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline size_t measure_lds(int ne, int ns, int M, size_t ts, bool ylds, bool flds) {
  return mal16((16 + (size_t)ns + M) * sizeof(double)) +
         (ylds ? mal16((size_t)ne * (ne / 2 + 1) * ts) : 0) +
         (flds ? mal16((size_t)ns * (ns + 1) * ts) : 0) + (size_t)(ne + 2 * ns) * sizeof(int32_t);
}

template <typename T, bool YLDS, bool FLDS>
__global__ __launch_bounds__(kMeasureThreads) void k_measure(Pools P,
                                                             const int32_t* __restrict__ wlist,
                                                             int slot, double* __restrict__ eloc,
                                                             T* __restrict__ O) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  const InstDev& I = P.inst[P.walker_inst[gw]];
  if (I.nproj) return;   // projected walkers: k_measure_proj
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, M = I.M, nup = I.nup;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x;
  const int ldf = ns + 1;

  unsigned char* q = smem;
  double* red = (double*)q;                     // 16
  double* hs = red + 16;                        // ns
  double* ths = hs + ns;                        // M
  q += mal16((16 + (size_t)ns + M) * sizeof(double));
  const T* Yglob = (const T*)P.Y + I.Y_off + lw * ne * ne;
  T* Ys = (T*)q;
  if (YLDS) q += mal16((size_t)ne * (ne / 2 + 1) * sizeof(T));
  const int ldy = nup + 1;   // padded rows of Yh avoid LDS bank conflicts
  T* fs = (T*)q;
  if (FLDS) q += mal16((size_t)ns * ldf * sizeof(T));
  int32_t* pos_s = (int32_t*)q;                 // ne
  int32_t* eidx = pos_s + ne;                   // 2ns

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  const T* A = table_of<T>(P, I.A_off);
  for (int v = tid; v < n2; v += blockDim.x) eidx[v] = -1;
  for (int l = tid; l < ns; l += blockDim.x) hs[l] = P.h[I.h_off + lw * ns + l];
  for (int hh = tid; hh < M; hh += blockDim.x) ths[hh] = P.theta[I.theta_off + lw * M + hh];
  if (YLDS)
    for (int e = tid; e < ne * nup; e += blockDim.x) {
      const int a = e / nup, bp = e - (e / nup) * nup;
      Ys[a * ldy + bp] = Yglob[(int64_t)a * ne + (a < nup ? nup : 0) + bp];
    }
  if (FLDS)
    for (int e = tid; e < ns * ns; e += blockDim.x) {
      const int i = e / ns, j = e - (e / ns) * ns;
      fs[i * ldf + j] = A[(int64_t)i * n2 + ns + j];
    }
  __syncthreads();
  for (int b = tid; b < ne; b += blockDim.x) {
    pos_s[b] = posg[b];
    eidx[posg[b]] = b;
  }
  __syncthreads();

  // Y[a][b] for electrons a, b of opposite spin
  auto yab = [&](int a, int b) -> T {
    return YLDS ? Ys[a * ldy + (b < nup ? b : b - nup)] : Yglob[(int64_t)a * ne + b];
  };
  // pair amplitude f(i, j) = A[i][Ns + j]
  auto fval = [&](int i, int j) -> T { return FLDS ? fs[i * ldf + j] : A[(int64_t)i * n2 + ns + j]; };
  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const double* Uv = P.U + I.site_off;
  const int32_t* nptr = P.nbr_ptr + I.nptr_off;
  const int32_t* nsite = P.nbr_site + I.nbr_off;
  const double* nt = P.nbr_t + I.nbr_off;
  const double* ra = P.rbm64 + I.rbm_a_off;
  const double* rW = P.rbm64 + I.rbm_W_off;

  double e = 0.0;
  for (int i = tid; i < ns; i += blockDim.x)
    if (eidx[i] >= 0 && eidx[i + ns] >= 0) e += Uv[i];
  const int deg = I.deg_max;
  for (int t = tid; t < ne * deg; t += blockDim.x) {
    const int a = t / deg, qn = t - (t / deg) * deg;
    const int Iold = pos_s[a];
    const int sigma = Iold >= ns ? 1 : 0;
    const int site_old = Iold - sigma * ns;
    const int s0 = nptr[site_old] + qn;
    if (s0 >= nptr[site_old + 1]) continue;
    const int site_new = nsite[s0];
    const int Inew = site_new + sigma * ns;
    if (eidx[Inew] >= 0) continue;
    // new row a of X is non-zero only on the opposite-spin electrons (Eq. AP-Pf)
    const T* Ya = YLDS ? Ys + a * ldy : Yglob + (int64_t)a * ne + (sigma ? 0 : nup);
    double s = 0.0;
    if (sigma == 0) {
#pragma unroll 8
      for (int bp = 0; bp < nup; ++bp)
        s += (double)Ya[bp] * (double)fval(site_new, pos_s[nup + bp] - ns);
    } else {
#pragma unroll 8
      for (int bp = 0; bp < nup; ++bp) s -= (double)Ya[bp] * (double)fval(pos_s[bp], site_new);
    }
    const double r_pf = -s;
    const int opp = (1 - sigma) * ns;
    double logc = G[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  G[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                  hs[site_old] - V[(int64_t)site_old * ns + site_new];
    if (M) {
      logc += 2.0 * (ra[Inew] - ra[Iold]);
      for (int hh = 0; hh < M; ++hh) {
        const double th = ths[hh];
        const double d = 2.0 * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
        logc += log2cosh(th + d) - log2cosh(th);
      }
    }
    e += -nt[s0] * r_pf * exp(logc);
  }
  e = block_sum(e, red);
  for (int hh = tid; hh < M; hh += blockDim.x) ths[hh] = tanh(ths[hh]);
  __syncthreads();
  const int64_t row = (int64_t)slot * I.W + lw;
  if (tid == 0) eloc[I.eloc_off + row] = e;

  T* Orow = O + I.O_off + row * I.ldO;
  const int32_t* fptr = P.fm_ptr + I.fm_ptr_off;
  slot_sums_any(I.nf, fptr[I.nf], fptr, P.fm + I.fm_off,
                [&](int pk) -> double {
                  const int ea = eidx[pk / ns], eb = eidx[pk % ns + ns];
                  return (ea >= 0 && eb >= 0) ? -(double)yab(ea, eb) : 0.0;
                },
                Orow);
  const int32_t* gptr = P.gm_ptr + I.gm_ptr_off;
  slot_sums_any(I.ng, gptr[I.ng], gptr, P.gm + I.gm_off,
                [&](int i) -> double { return (eidx[i] >= 0 && eidx[i + ns] >= 0) ? 1.0 : 0.0; },
                Orow + I.nf);
  const int32_t* vptr = P.vm_ptr + I.vm_ptr_off;
  slot_sums_any(I.nv, vptr[I.nv], vptr, P.vm + I.vm_off,
                [&](int pk) -> double {
                  const int i = pk / ns, j = pk % ns;
                  const int mi = (eidx[i] >= 0) + (eidx[i + ns] >= 0) - 1;
                  const int mj = (eidx[j] >= 0) + (eidx[j + ns] >= 0) - 1;
                  return (double)(mi * mj);
                },
                Orow + I.nf + I.ng);
  if (M) {
    T* Oa = Orow + I.nf + I.ng + I.nv;
    T* Ob = Oa + n2;
    T* OW = Ob + M;
    for (int v = tid; v < n2; v += blockDim.x) Oa[v] = (T)(eidx[v] >= 0 ? 1.0 : -1.0);
    for (int hh = tid; hh < M; hh += blockDim.x) Ob[hh] = (T)ths[hh];
    for (int64_t idx = tid; idx < (int64_t)M * n2; idx += blockDim.x) {
      const int hh = (int)(idx / n2), v = (int)(idx % n2);
      OW[idx] = (T)(eidx[v] >= 0 ? ths[hh] : -ths[hh]);
    }
  }
  for (int k = I.np + tid; k < I.ldO; k += blockDim.x) Orow[k] = T(0);
}

// Projected walkers (section 3.2.2, Eqs. momP and pointP): with
// c_p = w_p Pf(X(q_p(x))) / sum_q w_q Pf(X(q_q(x))),
//   hop ratio     R = sum_p c_p r_p times the correlator ratio, r_p from
//                 M_p^-1 and the mapped pair amplitudes as in the sweep;
//   f slot k      O = sum_p c_p sum over members (i, j) of M_p^-1[b][a] with
//                 a the up electron on q_p^-1(i) and b the down electron on
//                 q_p^-1(j) (Eq. DiffPf on each term);
//   g, v, RBM     as without projection.
// LDS: [red 16 | hs ns | ths M | c_p] doubles, then pos [N_e], eidx [2 N_s],
// maps and inverse maps [2 N_P N_s].
__host__ __device__ inline size_t measure_proj_lds(int ne, int ns, int M, int np) {
  return mal16((16 + (size_t)ns + M + np) * sizeof(double)) +
         (size_t)(ne + 2 * ns + 2 * (size_t)np * ns) * sizeof(int32_t);
}

template <typename T>
__global__ __launch_bounds__(kMeasureThreads) void k_measure_proj(
    Pools P, const int32_t* __restrict__ wlist, int slot, double* __restrict__ eloc,
    T* __restrict__ O) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, M = I.M, n = I.nup, np = I.nproj;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x;

  double* red = (double*)smem;                  // 16
  double* hs = red + 16;                        // ns
  double* ths = hs + ns;                        // M
  double* cp = ths + M;                         // np
  int32_t* pos_s = (int32_t*)(smem + mal16((16 + (size_t)ns + M + np) * sizeof(double)));
  int32_t* eidx = pos_s + ne;                   // 2ns
  int32_t* qm = eidx + n2;                      // [np][ns] maps, then [np][ns] inverses

  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  const T* Yw = (const T*)P.Y + I.Y_off + lw * I.Y_ld;
  const T* A = table_of<T>(P, I.A_off);
  for (int v = tid; v < n2; v += blockDim.x) eidx[v] = -1;
  for (int l = tid; l < ns; l += blockDim.x) hs[l] = P.h[I.h_off + lw * ns + l];
  for (int hh = tid; hh < M; hh += blockDim.x) ths[hh] = P.theta[I.theta_off + lw * M + hh];
  for (int e = tid; e < 2 * np * ns; e += blockDim.x) qm[e] = P.pmap[I.proj_off + e];
  if (tid == 0) {
    const double* lt = P.pterm + I.pterm_off + lw * 2 * np;
    const double* w = P.projw + I.projw_off;
    double lmax = -INFINITY;
    for (int p = 0; p < np; ++p)
      if (lt[np + p] != 0.0) lmax = fmax(lmax, lt[p]);
    double tot = 0.0;
    for (int p = 0; p < np; ++p) {
      const double c = lt[np + p] != 0.0 ? w[p] * lt[np + p] * exp(lt[p] - lmax) : 0.0;
      cp[p] = c;
      tot += c;
    }
    for (int p = 0; p < np; ++p) cp[p] /= tot;
  }
  __syncthreads();
  for (int b = tid; b < ne; b += blockDim.x) {
    pos_s[b] = posg[b];
    eidx[posg[b]] = b;
  }
  __syncthreads();

  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const double* Uv = P.U + I.site_off;
  const int32_t* nptr = P.nbr_ptr + I.nptr_off;
  const int32_t* nsite = P.nbr_site + I.nbr_off;
  const double* nt = P.nbr_t + I.nbr_off;
  const double* ra = P.rbm64 + I.rbm_a_off;
  const double* rW = P.rbm64 + I.rbm_W_off;

  double e = 0.0;
  for (int i = tid; i < ns; i += blockDim.x)
    if (eidx[i] >= 0 && eidx[i + ns] >= 0) e += Uv[i];
  const int deg = I.deg_max;
  for (int t = tid; t < ne * deg; t += blockDim.x) {
    const int a = t / deg, qn = t - (t / deg) * deg;
    const int Iold = pos_s[a];
    const int sigma = Iold >= ns ? 1 : 0;
    const int site_old = Iold - sigma * ns;
    const int s0 = nptr[site_old] + qn;
    if (s0 >= nptr[site_old + 1]) continue;
    const int site_new = nsite[s0];
    const int Inew = site_new + sigma * ns;
    if (eidx[Inew] >= 0) continue;
    const int ai = a - sigma * n;
    double r_pf = 0.0;
    for (int p = 0; p < np; ++p) {
      if (cp[p] == 0.0) continue;
      const int32_t* qp = qm + p * ns;
      const T* Mp = Yw + (int64_t)p * n * n;
      double s = 0.0;
      if (sigma == 0) {
        const T* Arow = A + (int64_t)qp[site_new] * n2 + ns;
        for (int b = 0; b < n; ++b)
          s += (double)Arow[qp[pos_s[n + b] - ns]] * (double)Mp[b * n + ai];
      } else {
        const int col = ns + qp[site_new];
        for (int i = 0; i < n; ++i)
          s += (double)Mp[ai * n + i] * (double)A[(int64_t)qp[pos_s[i]] * n2 + col];
      }
      r_pf += cp[p] * s;
    }
    const int opp = (1 - sigma) * ns;
    double logc = G[site_new] * (eidx[site_new + opp] >= 0 ? 1.0 : 0.0) -
                  G[site_old] * (eidx[site_old + opp] >= 0 ? 1.0 : 0.0) + hs[site_new] -
                  hs[site_old] - V[(int64_t)site_old * ns + site_new];
    if (M) {
      logc += 2.0 * (ra[Inew] - ra[Iold]);
      for (int hh = 0; hh < M; ++hh) {
        const double th = ths[hh];
        const double d = 2.0 * (rW[(int64_t)hh * n2 + Inew] - rW[(int64_t)hh * n2 + Iold]);
        logc += log2cosh(th + d) - log2cosh(th);
      }
    }
    e += -nt[s0] * r_pf * exp(logc);
  }
  e = block_sum(e, red);
  for (int hh = tid; hh < M; hh += blockDim.x) ths[hh] = tanh(ths[hh]);
  __syncthreads();
  const int64_t row = (int64_t)slot * I.W + lw;
  if (tid == 0) eloc[I.eloc_off + row] = e;

  T* Orow = O + I.O_off + row * I.ldO;
  const int32_t* fptr = P.fm_ptr + I.fm_ptr_off;
  slot_sums_any(I.nf, fptr[I.nf], fptr, P.fm + I.fm_off,
                [&](int pk) -> double {
                  const int i = pk / ns, j = pk % ns;
                  double s = 0.0;
                  for (int p = 0; p < np; ++p) {
                    if (cp[p] == 0.0) continue;
                    const int32_t* qi = qm + (np + p) * ns;
                    const int ea = eidx[qi[i]], eb = eidx[qi[j] + ns];
                    if (ea >= 0 && eb >= 0)
                      s += cp[p] * (double)Yw[(int64_t)p * n * n + (eb - n) * n + ea];
                  }
                  return s;
                },
                Orow);
  const int32_t* gptr = P.gm_ptr + I.gm_ptr_off;
  slot_sums_any(I.ng, gptr[I.ng], gptr, P.gm + I.gm_off,
                [&](int i) -> double { return (eidx[i] >= 0 && eidx[i + ns] >= 0) ? 1.0 : 0.0; },
                Orow + I.nf);
  const int32_t* vptr = P.vm_ptr + I.vm_ptr_off;
  slot_sums_any(I.nv, vptr[I.nv], vptr, P.vm + I.vm_off,
                [&](int pk) -> double {
                  const int i = pk / ns, j = pk % ns;
                  const int mi = (eidx[i] >= 0) + (eidx[i + ns] >= 0) - 1;
                  const int mj = (eidx[j] >= 0) + (eidx[j + ns] >= 0) - 1;
                  return (double)(mi * mj);
                },
                Orow + I.nf + I.ng);
  if (M) {
    T* Oa = Orow + I.nf + I.ng + I.nv;
    T* Ob = Oa + n2;
    T* OW = Ob + M;
    for (int v = tid; v < n2; v += blockDim.x) Oa[v] = (T)(eidx[v] >= 0 ? 1.0 : -1.0);
    for (int hh = tid; hh < M; hh += blockDim.x) Ob[hh] = (T)ths[hh];
    for (int64_t idx = tid; idx < (int64_t)M * n2; idx += blockDim.x) {
      const int hh = (int)(idx / n2), v = (int)(idx % n2);
      OW[idx] = (T)(eidx[v] >= 0 ? ths[hh] : -ths[hh]);
    }
  }
  for (int k = I.np + tid; k < I.ldO; k += blockDim.x) Orow[k] = T(0);
}

size_t measure_proj_lds_bytes(int ne, int ns, int M, int nproj) {
  return measure_proj_lds(ne, ns, M, nproj);
}

template <typename T>
void launch_measure_proj(const Pools& P, const int32_t* wlist, int n, int slot, double* eloc,
                         T* O, size_t lds_bytes, hipStream_t s) {
  if (n <= 0) return;
  if (lds_bytes > 65536)
    (void)hipFuncSetAttribute((const void*)&k_measure_proj<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  hipLaunchKernelGGL((k_measure_proj<T>), dim3(n), dim3(kMeasureThreads), lds_bytes, s, P, wlist,
                     slot, eloc, O);
}

template void launch_measure_proj<double>(const Pools&, const int32_t*, int, int, double*,
                                          double*, size_t, hipStream_t);
template void launch_measure_proj<float>(const Pools&, const int32_t*, int, int, double*, float*,
                                         size_t, hipStream_t);

template <typename T>
void launch_measure(const Pools& P, const int32_t* wlist, int n, int slot, double* eloc, T* O,
                    int max_ne, int max_ns, int max_M, hipStream_t s) {
  if (n <= 0) return;
  // Keep a workgroup's LDS small enough for several walkers per CU: the
  // opposite-spin half of Y is staged when it fits, the pair-amplitude table
  // (shared by every walker of an instance and L2-resident) only when small.
  const size_t budget = 64 * 1024;
  const bool ylds = measure_lds(max_ne, max_ns, max_M, sizeof(T), true, false) <= budget;
  const bool flds = (size_t)max_ns * (max_ns + 1) * sizeof(T) <= 16 * 1024 &&
                    measure_lds(max_ne, max_ns, max_M, sizeof(T), ylds, true) <= budget;
  const size_t sh = measure_lds(max_ne, max_ns, max_M, sizeof(T), ylds, flds);
#define MVMC_MEAS(YL, FL)                                                                       \
  do {                                                                                          \
    if (sh > 65536)                                                                             \
      (void)hipFuncSetAttribute((const void*)&k_measure<T, YL, FL>,                             \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);           \
    hipLaunchKernelGGL((k_measure<T, YL, FL>), dim3(n), dim3(kMeasureThreads), sh, s, P, wlist, \
                       slot, eloc, O);                                                          \
  } while (0)
  if (ylds && flds) MVMC_MEAS(true, true);
  else if (ylds) MVMC_MEAS(true, false);
  else if (flds) MVMC_MEAS(false, true);
  else MVMC_MEAS(false, false);
#undef MVMC_MEAS
}

template void launch_measure<double>(const Pools&, const int32_t*, int, int, double*, double*, int,
                                     int, int, hipStream_t);
template void launch_measure<float>(const Pools&, const int32_t*, int, int, double*, float*, int,
                                    int, int, hipStream_t);

}  // namespace mvmc
