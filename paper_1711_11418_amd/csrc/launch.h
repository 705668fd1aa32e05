// Host-side launchers for the kernels, one group per .hip file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mvmc {

// k_state.hip
void launch_expand(const Pools& P, const InstDev* inst_host, int n_inst, const double* params,
                   hipStream_t s);
void launch_draw_configs(const Pools& P, const int32_t* wlist, int n, uint64_t seed,
                         uint32_t attempt, hipStream_t s);
void launch_build_empty(const Pools& P, const int32_t* wlist, int n, int max_ns, hipStream_t s);
void launch_set_target(const Pools& P, uint64_t* target, int64_t W, int n_sweeps, hipStream_t s);
// int32 <-> int16 copies of the configurations (C-ABI form)
void launch_pos_narrow(const int32_t* src, int16_t* dst, int64_t n, hipStream_t s);
void launch_pos_widen(const int16_t* src, int32_t* dst, int64_t n, hipStream_t s);
// *out = index of the first non-finite x[i], or n when all are finite
void launch_first_nonfinite(const double* x, int64_t n, int64_t* out, hipStream_t s);

// k_refresh.hip: full double-precision X^-1, log|Pf|, sign, Jastrow field and
// RBM angles for the walkers in wlist.  T is the walker-matrix type.
// Refresh through the anti-parallel block M: X^-1 and Pf(X) from M^-1 and
// det M.  Route for a walker set: 1 one wavefront per walker (N_e <= 128),
// 2 a 16 x 16 thread tile per walker (N_e <= 256), 0 none (the generic skew
// elimination of k_refresh.hip).
int refresh_ap_route(int max_ne, int max_ns);
template <typename T>
void launch_refresh_ap(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                       int route, double sing_tol, int32_t* flags, hipStream_t s);
template <typename T>
void launch_refresh(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                    bool lds, double sing_tol, hipStream_t s);
size_t refresh_lds_bytes(int ne, int ns, bool lds);
// Same, only for walkers whose flag is set; clears the flag.
template <typename T>
void launch_refresh_if(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                       bool lds, int32_t* flags, hipStream_t s);
// double copy of a float array
void launch_widen(const float* src, double* dst, int64_t n, hipStream_t s);

// k_sweep.hip: n_prop Metropolis proposals per walker.
template <typename T>
void launch_sweep(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                  int max_ne, int max_ns, int max_M, bool lds, int nthreads,
                  TraceRec* trace, int64_t trace_cap, const uint64_t* trace_base,
                  const uint64_t* target, int32_t* needs_refresh, int R, hipStream_t s);
size_t sweep_lds_bytes(int ne, int ns, int M, bool lds, size_t tsize, int nthreads);

// k_sweep_ap.hip: the same proposals with only M^-1 (the anti-parallel block
// of X^-1) resident in LDS, rank-1 updates.
template <typename T>
void launch_sweep_ap(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                     int max_ne, int max_ns, int max_M, int nthreads, TraceRec* trace,
                     int64_t trace_cap, const uint64_t* trace_base, const uint64_t* target,
                     int32_t* needs_refresh, int R, int ex64, hipStream_t s);
size_t sweep_ap_lds_bytes(int ne, int ns, int M, size_t tsize, int nthreads);

// k_sweep_reg.hip: register-resident sweep, one wavefront per walker, groups
// of 4 walkers of one instance per workgroup (wlist padded with -1).
// Returns false when ne_max has no instantiation.
template <typename T>
bool launch_sweep_reg(const Pools& P, const int32_t* wlist, int n_groups, int ne_max, int max_ns,
                      int max_M, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
                      const uint64_t* trace_base, const uint64_t* target, int32_t* needs_refresh,
                      int R, int kref, int ex64, hipStream_t s);
size_t sweep_reg_lds_bytes(int ne_max, int ns, int M, size_t tsize, int wpb);
int sweep_reg_class(int ne, size_t tsize);   // register tier for ne, 0 = none

// k_sweep_queue.hip: one persistent launch over a cost-sorted item list
// (>= 0: anti-parallel-block walker; < 0: register-tier group -(item + 1) of
// `groups`, 4 walkers each), both tiers refreshing inside the launch.  head:
// one int of device memory, reset by the launch; lds_bytes: the largest
// sweep_queue_lds_bytes over the instances.  Returns false when the shapes
// have no instantiation (register tier above 64 electrons, anti-parallel
// block above 256).
template <typename T>
bool launch_sweep_queue(const Pools& P, const int32_t* items, int n_items, const int32_t* groups,
                        int32_t* head, int max_ne_reg, int max_ne_ap, size_t lds_bytes, bool full,
                        int n_cu, int cap, uint64_t seed, TraceRec* trace, int64_t trace_cap,
                        const uint64_t* trace_base, const uint64_t* target, int R, int ex64,
                        hipStream_t s);
// register blocks of the refresh tile for anti-parallel walkers of up to
// max_ne_ap electrons (0 none, -1 too large)
int sweep_queue_nb(int max_ne_ap);
// LDS of one instance's items: a register-tier instance (ne_reg > 0) or an
// anti-parallel one (ne_ap > 0)
size_t sweep_queue_lds_bytes(int ne_reg, int ne_ap, int ns, int M, size_t tsize);

// k_proj.hip: quantum-number projection (section 3.2.2) on the anti-parallel
// block.  Refresh: every term's M_p^-1, log|det M_p| and sign in double, the
// walker's sum over terms, Jastrow field and RBM angles (with flags, only
// flagged walkers, flags cleared).  Sweep: hopping proposals with every
// M_p^-1 in LDS (lds_bytes: the largest sweep_proj_lds_bytes of the list).
template <typename T>
void launch_refresh_proj(const Pools& P, const int32_t* wlist, int n, int max_ne, int max_ns,
                         double sing_tol, int32_t* flags, hipStream_t s);
size_t refresh_proj_lds_bytes(int ne, int ns);
template <typename T>
void launch_sweep_proj(const Pools& P, const int32_t* wlist, int n, int cap, uint64_t seed,
                       size_t lds_bytes, TraceRec* trace, int64_t trace_cap,
                       const uint64_t* trace_base, const uint64_t* target, int32_t* needs_refresh,
                       int R, hipStream_t s);
size_t sweep_proj_lds_bytes(int ne, int ns, int M, int nproj, size_t tsize);

// k_measure.hip: local energy and O_k rows for sample slot `slot` (projected
// walkers are skipped: launch_measure_proj covers them).
template <typename T>
void launch_measure(const Pools& P, const int32_t* wlist, int n, int slot, double* eloc, T* O,
                    int max_ne, int max_ns, int max_M, hipStream_t s);
template <typename T>
void launch_measure_proj(const Pools& P, const int32_t* wlist, int n, int slot, double* eloc,
                         T* O, size_t lds_bytes, hipStream_t s);
size_t measure_proj_lds_bytes(int ne, int ns, int M, int nproj);

// k_lanczos.hip: F(x, H) and F(x, H^2) of every listed walker into slot
// `slot` of f1 / f2 (eloc layout); moments, alpha_1 and E_1 per instance
// into out[k * 7 + 0..6].
template <typename T>
void launch_local_h2(const Pools& P, const int32_t* wlist, int n, int slot, double* f1,
                     double* f2, int max_ne, int max_ns, hipStream_t s);
size_t local_h2_lds_bytes(int ne, int ns);
void launch_lanczos_moments(const Pools& P, int n_inst, int n_used, const double* f1,
                            const double* f2, double* out, hipStream_t s);

// peak probes (k_probe.hip): 0 bf16 MFMA, 1 FP64 MFMA, 2 FP64 vector FMA
double probe_flops_per_wave_iter(int kind);
void launch_probe(int kind, float* out, int blocks, int iters, hipStream_t s);

}  // namespace mvmc
