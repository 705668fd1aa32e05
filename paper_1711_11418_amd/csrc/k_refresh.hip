// Full double-precision recomputation of a walker's state.
//
// <x|phi_Pf> is proportional to Pf(X), X_ab = A[I_a][I_b] (section 3.2.1).
// One workgroup per walker builds X and inverts it in place by block
// Gauss-Jordan elimination with 2x2 skew pivots.  A pivot block
// K = {i, j} with x = M[i][j] (taken from the current Schur complement) has
// P^-1 = [[0, -1/x], [1/x, 0]] and the in-place step
//     M_KK <- P^-1,   M_Kc <- P^-1 M_Kc,   M_rK <- -M_rK P^-1,
//     M_rc <- M_rc - M_rK P^-1 M_Kc          (r, c outside K),
// which after every index has been pivoted leaves X^-1 in M.  Because the
// Schur complement of a skew matrix is skew, the same pivots give
//     Pf(X) = sgn(pi) * prod_k x_k
// for the pivot order pi = (i1 j1 i2 j2 ...).  Partial pivoting: i is the
// first index not yet pivoted and j maximises |M[i][j]| over the rest.
//
// The same pass recomputes the Jastrow field h_l = sum_m v_lm (n_m - 1)
// (section 3.2.3) and the RBM angles theta = b + W sigma from scratch.
#include <float.h>

#include "launch.h"

namespace mvmc {

namespace {
constexpr int kRefreshThreads = 256;

// LDS carve-up shared by host sizing and device code.
struct RefreshLds {
  size_t M, vec, red, ints, total;
};
__host__ __device__ inline RefreshLds refresh_layout(int ne, int ns, bool lds) {
  RefreshLds L;
  L.M = lds ? (size_t)ne * ne * sizeof(double) : 0;
  L.vec = 4 * (size_t)ne * sizeof(double);
  L.red = 64 * sizeof(double);
  const int nint = 3 * ne + 2 * ns + 8;
  L.ints = (size_t)nint * sizeof(int32_t);
  L.total = L.M + L.vec + L.red + L.ints;
  return L;
}
}  // namespace

size_t refresh_lds_bytes(int ne, int ns, bool lds) { return refresh_layout(ne, ns, lds).total; }

template <typename T, bool LDS>
__global__ __launch_bounds__(kRefreshThreads) void k_refresh(Pools P,
                                                             const int32_t* __restrict__ wlist,
                                                             double sing_tol,
                                                             int32_t* __restrict__ flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  if (flags && !flags[gw]) return;
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns;
  const int64_t lw = gw - I.walker_off;
  const RefreshLds L = refresh_layout(ne, ns, LDS);
  double* M = LDS ? (double*)smem : P.Y64 + I.Y_off + lw * ne * ne;
  double* ri = (double*)(smem + L.M);
  double* rj = ri + ne;
  double* ci = rj + ne;
  double* cj = ci + ne;
  double* red = (double*)(smem + L.M + L.vec);
  int32_t* pos_s = (int32_t*)(smem + L.M + L.vec + L.red);
  int32_t* done = pos_s + ne;      // pivoted flags, later visited flags
  int32_t* order = done + ne;      // pivot sequence
  int32_t* occ = order + ne;       // 2*ns spin-orbital occupation
  int32_t* sc = occ + n2;          // scalars: [0] = i, [1] = j, [2] = singular

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int32_t* pos = P.pos + I.pos_off + lw * ne;
  for (int b = tid; b < ne; b += blockDim.x) {
    pos_s[b] = pos[b];
    done[b] = 0;
  }
  for (int v = tid; v < n2; v += blockDim.x) occ[v] = 0;
  if (tid == 0) sc[2] = 0;
  __syncthreads();
  for (int b = tid; b < ne; b += blockDim.x) occ[pos_s[b]] = 1;

  // X from the skew table; track max|X| as the scale of the singularity test
  const double* A = P.A64 + I.A_off;
  double amax = 0.0;
  for (int r = wid; r < ne; r += nw) {
    const double* Ar = A + (int64_t)pos_s[r] * n2;
    for (int c = lane; c < ne; c += 64) {
      const double v = Ar[pos_s[c]];
      M[r * ne + c] = v;
      amax = fmax(amax, fabs(v));
    }
  }
  // block max (reuse red)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  if (lane == 0) red[wid] = amax;
  __syncthreads();
  amax = 0.0;
  for (int w = 0; w < nw; ++w) amax = fmax(amax, red[w]);
  __syncthreads();

  double logabs = 0.0, sgn = 1.0, minpiv = DBL_MAX;
  int i = 0;
  for (int step = 0; step < ne / 2; ++step) {
    while (done[i]) ++i;   // uniform: every thread scans the same flags
    // j = argmax_{c not pivoted, c != i} |M[i][c]|; ties go to the lowest c
    double best = -1.0;
    int bj = ne;
    for (int c = tid; c < ne; c += blockDim.x) {
      if (!done[c] && c != i) {
        const double v = fabs(M[i * ne + c]);
        if (v > best) {
          best = v;
          bj = c;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int oj = __shfl_xor(bj, off, 64);
      if (ov > best || (ov == best && oj < bj)) {
        best = ov;
        bj = oj;
      }
    }
    if (lane == 0) {
      red[2 * wid] = best;
      red[2 * wid + 1] = (double)bj;
    }
    __syncthreads();
    best = -1.0;
    bj = ne;
    for (int w = 0; w < nw; ++w) {
      const double ov = red[2 * w];
      const int oj = (int)red[2 * w + 1];
      if (ov > best || (ov == best && oj < bj)) {
        best = ov;
        bj = oj;
      }
    }
    const int j = bj;
    if (j >= ne || !(best > sing_tol * amax)) {
      if (tid == 0) sc[2] = 1;
      break;   // uniform exit
    }
    const double x = M[i * ne + j];
    logabs += log(fabs(x));
    if (x < 0) sgn = -sgn;
    minpiv = fmin(minpiv, fabs(x));
    if (tid == 0) {
      order[2 * step] = i;
      order[2 * step + 1] = j;
    }
    for (int c = tid; c < ne; c += blockDim.x) {
      ri[c] = M[i * ne + c];
      rj[c] = M[j * ne + c];
      ci[c] = M[c * ne + i];
      cj[c] = M[c * ne + j];
    }
    __syncthreads();
    const double ix = 1.0 / x;
    for (int r = wid; r < ne; r += nw) {
      const bool rK = (r == i) || (r == j);
      const double cir = ci[r], cjr = cj[r];
      for (int c = lane; c < ne; c += 64) {
        const bool cK = (c == i) || (c == j);
        double v;
        if (!rK && !cK) {
          v = M[r * ne + c] - (cjr * ri[c] - cir * rj[c]) * ix;
        } else if (rK && !cK) {
          v = (r == i) ? -rj[c] * ix : ri[c] * ix;
        } else if (!rK) {
          v = (c == i) ? -cjr * ix : cir * ix;
        } else {
          v = (r == c) ? 0.0 : ((r == i) ? -ix : ix);
        }
        M[r * ne + c] = v;
      }
    }
    if (tid == 0) {
      done[i] = 1;
      done[j] = 1;
    }
    __syncthreads();
  }
  __syncthreads();
  const bool singular = sc[2] != 0;

  // sign of the pivot permutation: parity = sum over cycles of (length - 1)
  if (tid == 0 && !singular) {
    for (int b = 0; b < ne; ++b) done[b] = 0;
    int parity = 0;
    for (int b = 0; b < ne; ++b) {
      if (done[b]) continue;
      int c = b, len = 0;
      while (!done[c]) {
        done[c] = 1;
        c = order[c];
        ++len;
      }
      parity += len - 1;
    }
    if (parity & 1) sgn = -sgn;
    P.logpf[gw] = logabs;
    P.sgnpf[gw] = sgn;
    P.minpiv[gw] = minpiv / (amax > 0 ? amax : 1.0);
    P.status[gw] = 0;
    if (flags) flags[gw] = 0;
  } else if (tid == 0) {
    if (flags) flags[gw] = 0;
    P.logpf[gw] = -INFINITY;
    P.sgnpf[gw] = 0.0;
    P.minpiv[gw] = 0.0;
    P.status[gw] = 1;
  }
  if (!singular) {
    T* Y = (T*)P.Y + I.Y_off + lw * ne * ne;
    for (int e = tid; e < ne * ne; e += blockDim.x) Y[e] = (T)M[e];
  }

  // Jastrow field h_l = sum_m v_lm (n_m - 1)
  const double* V = P.V + I.V_off;
  double* h = P.h + I.h_off + lw * ns;
  for (int l = tid; l < ns; l += blockDim.x) {
    double s = 0.0;
    for (int m = 0; m < ns; ++m) s += V[l * ns + m] * (double)(occ[m] + occ[m + ns] - 1);
    h[l] = s;
  }
  // RBM angles theta_h = b_h + sum_v W_hv (2 n_v - 1)
  if (I.M) {
    const double* b = P.rbm64 + I.rbm_b_off;
    const double* Wm = P.rbm64 + I.rbm_W_off;
    double* th = P.theta + I.theta_off + lw * I.M;
    for (int hh = tid; hh < I.M; hh += blockDim.x) {
      double s = b[hh];
      const double* Wr = Wm + (int64_t)hh * n2;
      for (int v = 0; v < n2; ++v) s += Wr[v] * (double)(2 * occ[v] - 1);
      th[hh] = s;
    }
  }
}

template <typename T>
static void refresh_impl(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                         bool lds, double sing_tol, int32_t* flags, hipStream_t s) {
  if (n <= 0) return;
  // up to 128 electrons per spin: the anti-parallel block route, with the
  // block in registers (one wavefront per walker, or a 16 x 16 thread tile)
  if (const int route = refresh_ap_route(max_ne, max_ns)) {
    launch_refresh_ap<T>(P, wlist, n, max_ne, max_ns, route, sing_tol, flags, s);
    return;
  }
  const size_t sh = refresh_lds_bytes(max_ne, max_ns, lds);
  if (lds) {
    if (sh > 65536)
      (void)hipFuncSetAttribute((const void*)&k_refresh<T, true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh<T, true>), dim3(n), dim3(kRefreshThreads), sh, s, P, wlist,
                       sing_tol, flags);
  } else {
    if (sh > 65536)
      (void)hipFuncSetAttribute((const void*)&k_refresh<T, false>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    hipLaunchKernelGGL((k_refresh<T, false>), dim3(n), dim3(kRefreshThreads), sh, s, P, wlist,
                       sing_tol, flags);
  }
}

template <typename T>
void launch_refresh(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns, bool lds,
                    double sing_tol, hipStream_t s) {
  refresh_impl<T>(P, wlist, n, max_ne, max_ns, lds, sing_tol, nullptr, s);
}

template <typename T>
void launch_refresh_if(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                       bool lds, int32_t* flags, hipStream_t s) {
  refresh_impl<T>(P, wlist, n, max_ne, max_ns, lds, 0.0, flags, s);
}

__global__ void k_widen(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

void launch_widen(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)nb), dim3(256), 0, s, src, dst, n);
}

template void launch_refresh<double>(const Pools&, const int32_t*, int, int, int, bool, double,
                                     hipStream_t);
template void launch_refresh<float>(const Pools&, const int32_t*, int, int, int, bool, double,
                                    hipStream_t);
template void launch_refresh_if<double>(const Pools&, const int32_t*, int, int, int, bool,
                                        int32_t*, hipStream_t);
template void launch_refresh_if<float>(const Pools&, const int32_t*, int, int, int, bool, int32_t*,
                                       hipStream_t);

}  // namespace mvmc
