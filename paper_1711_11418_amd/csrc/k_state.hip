// Parameter expansion and walker-state construction.
//
// Expansion (section 3.2.1, Eq. AP-Pf; section 3.2.3): the parameter vector
// alpha is mapped through the Orbital/Gutzwiller/Jastrow index maps onto
//   A[(i,up),(j,dn)] = f_ij,  A[(j,dn),(i,up)] = -f_ij   (A = F - F^T),
//   v_ij (zero diagonal), g_i, and the RBM a, b, W copies.
// A is kept in double and in single precision; the sweep reads the one that
// matches its arithmetic.
#include <algorithm>

#include "launch.h"

namespace mvmc {

__global__ void k_expand(Pools P, const double* __restrict__ params) {
  const InstDev& I = P.inst[blockIdx.y];
  const int ns = I.ns, n2 = 2 * ns;
  const double* p = params + I.param_off;
  const int32_t* fidx = P.fidx + I.V_off;
  const int32_t* vidx = P.vidx + I.V_off;
  const int32_t* gidx = P.gidx + I.site_off;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t e = t0; e < (int64_t)n2 * n2; e += stride) {
    const int r = (int)(e / n2), c = (int)(e % n2);
    double v = 0.0;
    if (r < ns && c >= ns) {
      const int k = fidx[r * ns + (c - ns)];
      v = k >= 0 ? p[k] : 0.0;
    } else if (r >= ns && c < ns) {
      const int k = fidx[c * ns + (r - ns)];
      v = k >= 0 ? -p[k] : 0.0;
    }
    P.A64[I.A_off + e] = v;
    P.A32[I.A_off + e] = (float)v;
  }
  for (int64_t e = t0; e < (int64_t)ns * ns; e += stride) {
    const int r = (int)(e / ns), c = (int)(e % ns);
    const int k = vidx[e];
    P.V[I.V_off + e] = (k >= 0 && r != c) ? p[I.nf + I.ng + k] : 0.0;
  }
  for (int64_t e = t0; e < ns; e += stride) {
    const int k = gidx[e];
    P.G[I.site_off + e] = k >= 0 ? p[I.nf + k] : 0.0;
  }
  if (I.M) {
    const int64_t nr = (int64_t)n2 + I.M + (int64_t)I.M * n2;
    const double* pr = p + I.nf + I.ng + I.nv;
    const int64_t nab = (int64_t)n2 + I.M;
    for (int64_t e = t0; e < nr; e += stride) {
      P.rbm64[I.rbm_a_off + e] = pr[e];
      P.rbm32[I.rbm_a_off + e] = (float)pr[e];
      // transposed copy: W^T[v][h] = W[h][v]
      int64_t et = e;
      if (e >= nab) {
        const int64_t w = e - nab, hh = w / n2, v = w - hh * n2;
        et = nab + v * I.M + hh;
      }
      P.rbmT64[I.rbm_a_off + et] = pr[e];
      P.rbmT32[I.rbm_a_off + et] = (float)pr[e];
    }
  }
}

void launch_expand(const Pools& P, const InstDev* inst_host, int n_inst, const double* params,
                   hipStream_t s) {
  int64_t mx = 0;
  for (int i = 0; i < n_inst; ++i) {
    const int64_t n2 = 2 * (int64_t)inst_host[i].ns;
    int64_t e = n2 * n2;
    const int64_t r = inst_host[i].M ? n2 + inst_host[i].M + inst_host[i].M * n2 : 0;
    if (r > e) e = r;
    if (e > mx) mx = e;
  }
  int nb = (int)ceil_div<int64_t>(mx, 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_expand, dim3(nb, n_inst), dim3(256), 0, s, P, params);
}

// Uniform random configuration: a partial Fisher-Yates shuffle of the sites
// for each spin, drawn from Philox stream tag 1 with counter
// (draw index, attempt, walker, 1); sites are stored in ascending order.
__global__ void k_draw_configs(Pools P, const int32_t* __restrict__ wlist, uint64_t seed,
                               uint32_t attempt) {
  extern __shared__ int32_t sh[];
  const int gw = wlist[blockIdx.x];
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ns = I.ns;
  int32_t* list = sh;          // ns
  int32_t* mark = sh + ns;     // ns
  int32_t* pos = P.pos + I.pos_off + (int64_t)(gw - I.walker_off) * I.ne;
  if (threadIdx.x == 0) {
    uint32_t k_draw = 0;
    for (int sigma = 0; sigma < 2; ++sigma) {
      const int nsig = sigma ? I.ndn : I.nup;
      for (int s2 = 0; s2 < ns; ++s2) {
        list[s2] = s2;
        mark[s2] = 0;
      }
      uint4 r = make_uint4(0, 0, 0, 0);
      for (int k = 0; k < nsig; ++k) {
        const int word = k_draw & 3;
        if (word == 0) r = draw(seed, ((uint64_t)attempt << 32) | (k_draw >> 2), gw, 1u);
        const uint32_t rv = word == 0 ? r.x : word == 1 ? r.y : word == 2 ? r.z : r.w;
        ++k_draw;
        const int j = k + scaled(rv, ns - k);
        const int tmp = list[k];
        list[k] = list[j];
        list[j] = tmp;
        mark[list[k]] = 1;
      }
      int e = sigma ? I.nup : 0;
      for (int s2 = 0; s2 < ns; ++s2)
        if (mark[s2]) pos[e++] = s2 + sigma * ns;
      k_draw = (k_draw + 3) & ~3u;   // next spin starts on a fresh Philox block
    }
  }
}

void launch_draw_configs(const Pools& P, const int32_t* wlist, int n, uint64_t seed,
                         uint32_t attempt, hipStream_t s) {
  if (n <= 0) return;
  // dynamic LDS sized for the largest lattice (bounded at init)
  hipLaunchKernelGGL(k_draw_configs, dim3(n), dim3(64), 2 * 1024 * sizeof(int32_t), s, P, wlist,
                     seed, attempt);
}

// Empty-site lists in ascending site order, one list per spin.
__global__ void k_build_empty(Pools P, const int32_t* __restrict__ wlist) {
  extern __shared__ int32_t occ[];
  const int gw = wlist[blockIdx.x];
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ns = I.ns;
  const int64_t lw = gw - I.walker_off;
  const int32_t* pos = P.pos + I.pos_off + lw * I.ne;
  for (int v = threadIdx.x; v < 2 * ns; v += blockDim.x) occ[v] = 0;
  __syncthreads();
  for (int b = threadIdx.x; b < I.ne; b += blockDim.x) occ[pos[b]] = 1;
  __syncthreads();
  if (threadIdx.x < 2) {
    const int sigma = threadIdx.x;
    int32_t* emp = P.empty + I.empty_off + (lw * 2 + sigma) * ns;
    int k = 0;
    for (int s2 = 0; s2 < ns; ++s2)
      if (!occ[s2 + sigma * ns]) emp[k++] = s2;
    for (; k < ns; ++k) emp[k] = -1;
  }
}

// target[w] = cnt[w] + n_sweeps * N_e(instance of w): the proposal index at
// which this call's sweeps end for every walker.
__global__ void k_set_target(Pools P, uint64_t* __restrict__ target, int64_t W, int n_sweeps) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  target[w] = P.cnt[w] + (uint64_t)n_sweeps * (uint64_t)P.inst[P.walker_inst[w]].ne;
}

void launch_set_target(const Pools& P, uint64_t* target, int64_t W, int n_sweeps, hipStream_t s) {
  hipLaunchKernelGGL(k_set_target, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s, P, target,
                     W, n_sweeps);
}

// Index of the first non-finite entry of x[0, n) (n when every entry is
// finite): one workgroup, a fixed-order minimum.
__global__ void k_first_nonfinite(const double* __restrict__ x, int64_t n, int64_t* out) {
  __shared__ int64_t red[256];
  int64_t first = n;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    if (!isfinite(x[i])) {
      first = i;
      break;
    }
  red[threadIdx.x] = first;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w && red[threadIdx.x + w] < red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

void launch_first_nonfinite(const double* x, int64_t n, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_first_nonfinite, dim3(1), dim3(256), 0, s, x, n, out);
}

// Walker configurations cross the C ABI as int16 spin-orbital indices
// (2 N_s <= 2048); the walker pools keep int32.
__global__ void k_pos_narrow(const int32_t* __restrict__ src, int16_t* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (int16_t)src[i];
}
__global__ void k_pos_widen(const int16_t* __restrict__ src, int32_t* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (int32_t)src[i];
}

void launch_pos_narrow(const int32_t* src, int16_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pos_narrow, dim3(nb), dim3(256), 0, s, src, dst, n);
}
void launch_pos_widen(const int16_t* src, int32_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pos_widen, dim3(nb), dim3(256), 0, s, src, dst, n);
}

void launch_build_empty(const Pools& P, const int32_t* wlist, int n, int max_ns, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_build_empty, dim3(n), dim3(64), 2 * max_ns * sizeof(int32_t), s, P, wlist);
}

}  // namespace mvmc
