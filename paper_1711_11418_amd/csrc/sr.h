// Device-side structures and launchers for the stochastic-reconfiguration kernels.
#pragma once

#include "common.h"

namespace mvmc {

constexpr int kRowChunk = 512;   // rows per partial of the column passes

// per-instance scalar slots (scal[inst * kScal + slot])
enum : int {
  kEbar = 0, kEvar = 1, kRho = 2, kRhoNew = 3, kPw = 4, kBeta = 5, kThresh = 6, kDone = 7,
  kIters = 8, kFlag = 9, kEerr = 10, kScal = 16
};

struct SrInst {
  int64_t np, ldO, rows;          // parameters, O stride, samples used in this SR step
  int64_t walkers;                // independent chains; sample row = slot * walkers + walker
  int64_t O_off, S_off, eloc_off, param_off;
  int64_t colpart_off, syrkpart_off, chol_off, split_off;
  int64_t split_rows;             // rows per bf16 array (multiple of 32; zero past rows)
  int64_t split_ld;               // parameter stride of the bf16 arrays (>= ldO, covers every tile)
  int32_t ksplit;                 // sample split of the 64-tile split-bf16 S kernel
  int32_t sb;                     // 0: 64-tile kernel; 2..4: direct-to-LDS tiles of side 64 sb
  int32_t nfull;                  // direct-to-LDS tiles computed whole (the first nfull)
  int32_t tail_ks;                // sample parts of each remaining (tail) tile
  int32_t wide64;                 // 1: FP64 S by 128 x 128 tiles (nfull whole, the rest in tail_ks parts)
  int32_t pad0;
};

// Launch shape of the split-bf16 S build over all instances: whether any
// instance takes the 64-tile kernel, and per tile side 64 b the largest
// unit count (grid) and tail-tile count.
struct SyrkLaunch {
  bool any64;
  int units[5];
  int tail[5];
};

// bf16 split layout: element (sample m, parameter k) of the hi (or lo) array
// at ((m / 8) * split_ld + k) * 8 + m % 8, so the eight samples of one k-group
// of a parameter are one 16-byte vector (an MFMA operand).
__host__ __device__ inline int64_t split_index(int64_t m, int64_t k, int64_t ld) {
  return ((m >> 3) * ld + k) * 8 + (m & 7);
}

struct SrArgs {
  const SrInst* inst;
  const double* eloc;
  double* obar;
  double* sdiag;
  double* scal;
  double* colpart;
  double* syrkpart;
  double* chol;
  double* x;
  double* r;
  double* p;
  double* w;
  double* t;
  double* shift;
  double* mask;
  double* dotpart;                // [inst][kDotParts] partial dot products
};

constexpr int kDotParts = 256;    // most partial sums of one dot product

// bfloat16 with round-to-nearest-even (NaN kept quiet).
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  if ((v.u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((v.u >> 16) | 0x40u);
  v.u += 0x7fffu + ((v.u >> 16) & 1u);
  return (uint16_t)(v.u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  union { float f; uint32_t u; } v;
  v.u = (uint32_t)h << 16;
  return v.f;
}

void sr_estats(const SrArgs& A, int n_inst, hipStream_t s);
template <typename T>
void sr_colstats(const SrArgs& A, T* O, uint16_t* split, double* g, int n_inst, int64_t max_ld,
                 int64_t max_rows, hipStream_t s);
template <typename T, typename TS>
void sr_syrk_vec(const SrArgs& A, const T* O, TS* S, int n_inst, int64_t max_np, int max_ksplit,
                 bool any_wide, bool any_narrow, int wide_units, int wide_tail,
                 hipStream_t s);
// split-bf16 (hi*hi + hi*lo + lo*hi) MFMA S build, FP32 accumulation
void sr_syrk_bf16x3(const SrArgs& A, const uint16_t* split, float* S, int n_inst, int64_t max_np,
                    int max_ksplit, const SyrkLaunch& L, hipStream_t s);
template <typename TS>
void sr_cholesky_solve(const SrArgs& A, const TS* S, const double* g, double eps_rel, double eps_abs,
                       double freeze, int n_inst, int64_t max_np, hipStream_t s);
template <typename T>
void sr_cg_begin(const SrArgs& A, const double* g, double eps_rel, double eps_abs, double freeze,
                 double eps, int n_inst, int64_t max_np, hipStream_t s);
template <typename T>
void sr_cg_iter(const SrArgs& A, const T* O, int iter, int n_inst, int64_t max_np, int64_t max_rows,
                hipStream_t s);
void sr_apply(const SrArgs& A, double dtau, double* params, double* dparams, int n_inst,
              int64_t max_np, hipStream_t s);

}  // namespace mvmc
