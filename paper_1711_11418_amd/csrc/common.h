// Shared device-side definitions for the MI355X (gfx950) many-variable VMC library.
//
// Notation follows arXiv:1711.11418: Ns sites, N_e electrons, spin-orbital
// I = i + Ns*sigma (section 3.2.1); X is the N_e x N_e skew-symmetric matrix
// X_ab = A[I_a][I_b] with A = F - F^T; Y = X^-1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave.h"

namespace mvmc {

constexpr int kWave = 64;

// Per-instance table, resident in device memory.  Every *_off is an element
// offset into the matching pool (see workspace layout in api.cpp).
struct InstDev {
  int32_t ns, nup, ndn, ne;       // sites, electrons per spin, total electrons
  int32_t nf, ng, nv, M;          // parameter counts; M = RBM hidden units
  int32_t W, np, ldO, deg_max;    // walkers, parameters, O row stride, max lattice degree
  int32_t sweep_lds, refresh_lds; // 1 = matrix resident in LDS for that kernel
  int32_t nproj, pad0;            // quantum-number projection terms N_P (0 = none)
  int64_t walker_off;             // first global walker id
  int64_t param_off;              // offset into the concatenated parameter vector
  int64_t O_off, S_off, eloc_off; // caller buffers
  int64_t A_off;                  // skew table pool, (2Ns)^2 each (A64 and A32)
  int64_t V_off;                  // Jastrow v_ij, Ns^2 doubles
  int64_t site_off;               // per-site pools (G, U, gidx), Ns each
  int64_t nptr_off;               // neighbour CSR row pointers, Ns+1 each
  int64_t nbr_off;                // neighbour pools (site, t), 2*nbonds each
  int64_t fm_ptr_off, fm_off;     // f-slot members: CSR over slots of packed i*Ns+j
  int64_t gm_ptr_off, gm_off;     // g-slot members: CSR of sites
  int64_t vm_ptr_off, vm_off;     // v-slot members: CSR of packed i*Ns+j, i<j
  int64_t rbm_a_off, rbm_b_off, rbm_W_off;   // RBM pools (a: 2Ns, b: M, W: M*2Ns)
  int64_t Y_off;                  // walker-matrix pool: W * Y_ld
  int64_t Y_ld;                   // ne*ne, or max(ne*ne, nproj n^2) with a projection
  int64_t proj_off;               // pmap pool: maps q_p [nproj][ns], then inverses [nproj][ns]
  int64_t projw_off;              // projw pool: weights w_p [nproj]
  int64_t pterm_off;              // pterm pool, per walker: log|det M_p| [nproj], sign [nproj]
  int64_t pos_off;                // W * ne
  int64_t empty_off;              // W * 2*Ns  ([w][sigma][Ns], first Ns-N_sigma used)
  int64_t h_off;                  // W * Ns   (Jastrow field, double)
  int64_t theta_off;              // W * M    (RBM angles, double)
  int64_t chol_off;               // FP64 factor pool: np*np
  int64_t split_off;              // bf16 hi/lo pool: rows*ldO each
  int64_t rows;                   // samples per SR step = n_slots * W
};

// Global device pools shared by every kernel.
struct Pools {
  const InstDev* inst;
  const int32_t* walker_inst;      // global walker -> instance
  double* A64;
  float* A32;
  double* V;
  double* G;
  double* U;
  int32_t* nbr_ptr;
  int32_t* nbr_site;
  double* nbr_t;
  int32_t* fidx;                   // [Ns*Ns] per instance (V_off), -1 = fixed zero
  int32_t* vidx;                   // [Ns*Ns] per instance (V_off)
  int32_t* gidx;                   // [Ns] per instance (site_off)
  int32_t* fm_ptr;
  int32_t* fm;
  int32_t* gm_ptr;
  int32_t* gm;
  int32_t* vm_ptr;
  int32_t* vm;
  double* rbm64;                   // a, b, W in double
  float* rbm32;                    // same, single precision
  double* rbmT64;                  // a, b, W^T ([2Ns][M]) in double
  float* rbmT32;                   // same, single precision
  void* Y;                         // double or float walker matrices
  double* Y64;                     // double scratch for refreshes that do not fit LDS
  int32_t* pos;
  int32_t* empty;
  double* h;
  double* theta;
  uint64_t* cnt;                   // Philox proposal counter per walker
  uint64_t* upd;                   // applied updates per walker since the context's creation
  int64_t* accepted;
  double* logpf;
  double* sgnpf;
  double* minpiv;
  int32_t* status;
  // non-finite ratio guard per walker: 0 clear; 1 a ratio was not finite and
  // the walker waits for a double refresh before retrying that proposal;
  // 2 still not finite after the refresh: the walker stops
  int32_t* guard;
  int32_t* pmap;                   // projection site maps and their inverses
  double* projw;                   // projection weights
  double* pterm;                   // per-term log|det M_p| and sign of projected walkers
  // refresh_every counts applied updates (1) or proposals (0)
  int32_t refresh_upd;
  int32_t pad_pools;
};

enum : int32_t { kGuardClear = 0, kGuardPending = 1, kGuardFailed = 2 };

// One record per proposal when tracing is on.
struct TraceRec {
  int64_t n;          // proposal index of the walker
  int32_t walker;     // global walker id
  int32_t a;          // electron (the up electron of an exchange)
  int32_t i_new;      // proposed spin-orbital of a (-1: no move possible)
  int32_t accepted;
  double ratio;       // psi(x')/psi(x) including correlators
  int32_t b;          // down electron of an exchange, -1 for a hop
  int32_t pad;
};

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 32x32->64 products
// per round, Weyl bump of the key between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t n, uint32_t walker, uint32_t tag) {
  return philox4x32_10(make_uint4((uint32_t)n, (uint32_t)(n >> 32), walker, tag),
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Same draw with the key words passed through an opaque scalar move, so a
// caller inside a long loop recomputes the ten round keys instead of keeping
// all of them live in scalar registers.
__device__ __forceinline__ uint4 draw_lean(uint64_t seed, uint64_t n, uint32_t walker,
                                           uint32_t tag) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  asm volatile("" : "+s"(k0), "+s"(k1));
  return philox4x32_10(make_uint4((uint32_t)n, (uint32_t)(n >> 32), walker, tag), k0, k1);
}

// Multiply-shift map of a 32-bit word onto {0..n-1}.
__device__ __forceinline__ int scaled(uint32_t r, int n) {
  return (int)(((uint64_t)r * (uint64_t)n) >> 32);
}

// 53-bit uniform in [0,1), exact in binary64.
__device__ __forceinline__ double uniform53(uint32_t r2, uint32_t r3) {
  return ((double)(r2 >> 5) * 67108864.0 + (double)(r3 >> 6)) * (1.0 / 9007199254740992.0);
}

// log(2 cosh x), stable for large |x|.
__device__ __forceinline__ double log2cosh(double x) {
  const double ax = fabs(x);
  return ax + log1p(exp(-2.0 * ax));
}
__device__ __forceinline__ float log2cosh(float x) {
  const float ax = fabsf(x);
  return ax + log1pf(__expf(-2.0f * ax));
}

// ------------------------------------------------------------ reductions
// Sum over the 64 lanes of a fully active wavefront, the total in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
// doubles through the DPP row operations and a scalar read-back (each
// __shfl_xor step is an LDS permute round trip)
template <>
__device__ __forceinline__ double wave_sum<double>(double v) {
  return wave::wave_total(v);
}

// Block-wide sum of two values; every thread gets the totals.  `red` holds
// 2 * (blockDim/64) doubles of LDS.  Contains two barriers.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  if (nw == 1) return;
  if (lane == 0) {
    red[2 * wid] = a;
    red[2 * wid + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += red[2 * w];
    b += red[2 * w + 1];
  }
  __syncthreads();
}

__device__ __forceinline__ double block_sum(double a, double* red) {
  double b = 0.0;
  block_sum2(a, b, red);
  return a;
}

template <typename T>
__host__ __device__ inline T ceil_div(T a, T b) { return (a + b - 1) / b; }

}  // namespace mvmc
