// Host runtime of libmvmc: argument checks, workspace planning, walker
// buckets, and the call sequence behind each entry point of include/mvmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mvmc.h"
#include "launch.h"
#include "sr.h"

using namespace mvmc;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 152 * 1024;   // per-workgroup LDS budget used for residency
constexpr int kMaxSites = 1024;
constexpr int kMaxElec = 2048;
constexpr int kTimingCats = 6;
constexpr int kRegWpb = 4;   // walkers per workgroup of the register sweep
constexpr int kMaxShiftEscalations = 4;   // Cholesky retries with eps_rel x 10 each
constexpr int kTailUnitsMax = 512;        // split-bf16 S: sample parts of tail tiles, all together
constexpr int kWideTile = 128;            // FP64 wide S: tile side of k_syrk_f64_wide
constexpr int kWideTailUnits = 512;       // FP64 wide S: sample parts of tail tiles, all together
constexpr int kMaxTileSb = 4;             // largest direct-to-LDS S tile: 64 * 4

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------- planning
struct Pool {
  size_t off = 0, bytes = 0;
};

struct Plan {
  std::vector<InstDev> inst;
  std::vector<SrInst> sr;
  std::vector<int> reg_class;     // register-sweep tier per instance (0 = LDS/HBM kernel)
  std::vector<int> sweep_nt;      // threads of the LDS/HBM sweep kernel per instance
  std::vector<char> sweep_ap;     // 1 = anti-parallel-block sweep (M^-1 alone in LDS)
  bool any_proj = false;          // some instance has a quantum-number projection
  size_t proj_sweep_lds = 0, proj_measure_lds = 0;   // largest needs over projected instances
  int bad_variant = -1;           // instance a forced sweep variant does not fit
  bool exchange = false;          // exchange updates on (variants 0 and 7-9 only)
  bool queue = false;             // one persistent sweep launch (variants 0 and 9 only)
  // pools (byte offsets into the workspace)
  Pool inst_p, srinst_p, walker_inst, lists, A64, A32, V, fidx, vidx, G, U, gidx, nbr_ptr,
      nbr_site, nbr_t, fm_ptr, fm, gm_ptr, gm, vm_ptr, vm, rbm64, rbm32, rbmT64, rbmT32, Y, Y64,
      pos, empty, h,
      theta, pmap, projw, pterm, cnt, upd, target, needs_refresh, accepted, logpf, sgnpf, minpiv, status, guard, chk, lz,
      dotpart,
      trace_base,
      obar, sdiag, x, r, p, w, t, shift, mask, scal, colpart, syrkpart, chol, split;
  size_t total = 0;
  int64_t W = 0, np = 0, eloc = 0, O_elems = 0, S_elems = 0, Y_elems = 0;
  int max_ne = 0, max_ns = 0, max_M = 0, max_ksplit = 1;
  int64_t max_np = 0, max_ld = 0, max_rows = 0, max_sld = 0;
  bool need_Y64 = false;
  size_t tsize = 8;
};

struct HostInst {
  std::vector<int32_t> f_idx, v_idx, g_idx;
  std::vector<int32_t> nbr_ptr, nbr_site;
  std::vector<double> nbr_t, U;
  std::vector<int32_t> fm_ptr, fm, gm_ptr, gm, vm_ptr, vm;
};

struct Err {
  int code = MVMC_OK;
  std::string msg;
};

Err fail(int code, const char* fmt, ...) {
  Err e;
  e.code = code;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  e.msg = buf;
  return e;
}

int sweep_threads_for(const mvmc_config& c, int ne) {
  if (c.sweep_threads) return c.sweep_threads;
  return ne <= 48 ? 64 : (ne <= 96 ? 128 : 256);
}

// Parameter sets wide enough for one wavefront per 128 x 128 tile of S to
// fill the GPU without splitting the sample sum (at least 512 tiles in the
// upper triangle).
static bool wide_params(int64_t np) {
  const int64_t nt = (np + 127) / 128;
  return nt * (nt + 1) / 2 >= 512;
}

// Parameter stride of the bf16 split arrays: every direct-to-LDS tile side
// (128, 192, 256) reads whole tiles without leaving the row.
static int64_t split_ld_for(int64_t np, int64_t ldO) {
  int64_t ld = ldO;
  for (int b = 2; b <= kMaxTileSb; ++b) ld = std::max(ld, (np + 64 * b - 1) / (64 * b) * (64 * b));
  return ld;
}

// Tile side 64 sb of the direct-to-LDS S kernel (0: the 64-tile kernel) and
// the split of the tiles past the last full round over n_slots workgroup
// slots into sample parts, so the last round is as full as the others.
static void set_tiles(SrInst& S, int sb, int n_cu) {
  S.sb = sb;
  S.nfull = 0;
  S.tail_ks = 1;
  if (!sb && S.wide64) {   // FP64 wide tiles: two workgroups per compute unit
    const int64_t nt = (S.np + kWideTile - 1) / kWideTile, ntl = nt * (nt + 1) / 2;
    const int64_t slots = 2 * (int64_t)std::max(n_cu, 1);
    const int64_t rem = ntl % slots;
    S.nfull = (int32_t)ntl;
    if (rem) {
      int64_t ks = std::min<int64_t>(8, slots / rem);
      while (ks > 1 && rem * ks > kWideTailUnits) --ks;
      if (ks >= 2) {
        S.nfull = (int32_t)(ntl - rem);
        S.tail_ks = (int32_t)ks;
      }
    }
    return;
  }
  if (!sb) return;
  const int64_t T = 64 * sb, nt = (S.np + T - 1) / T, ntl = nt * (nt + 1) / 2;
  const int64_t slots = (int64_t)std::max(n_cu, 1) * (sb == 2 ? 2 : 1);
  const int64_t rem = ntl % slots;
  S.nfull = (int32_t)ntl;
  if (rem) {
    int64_t ks = std::min<int64_t>(8, slots / rem);
    while (ks > 1 && rem * ks > kTailUnitsMax) --ks;
    if (ks >= 2) {
      S.nfull = (int32_t)(ntl - rem);
      S.tail_ks = (int32_t)ks;
    }
  }
}

Err validate(const mvmc_config* c) {
  if (!c) return fail(MVMC_E_ARG, "config is NULL");
  if (c->precision != MVMC_FP64 && c->precision != MVMC_MIXED)
    return fail(MVMC_E_ARG, "precision must be MVMC_FP64 or MVMC_MIXED");
  if (c->refresh_every < 0) return fail(MVMC_E_ARG, "refresh_every < 0");
  if (c->refresh_unit != MVMC_REFRESH_PROPOSALS && c->refresh_unit != MVMC_REFRESH_UPDATES)
    return fail(MVMC_E_ARG, "refresh_unit must be MVMC_REFRESH_PROPOSALS or MVMC_REFRESH_UPDATES");
  if (c->n_instances < 1 || !c->inst) return fail(MVMC_E_ARG, "need at least one instance");
  if (c->n_slots < 1) return fail(MVMC_E_ARG, "n_slots must be >= 1");
  if (c->solver != MVMC_SOLVE_CHOL && c->solver != MVMC_SOLVE_CG)
    return fail(MVMC_E_ARG, "solver must be MVMC_SOLVE_CHOL or MVMC_SOLVE_CG");
  if (c->solver == MVMC_SOLVE_CHOL && !c->build_s)
    return fail(MVMC_E_ARG, "the Cholesky solver needs build_s = 1");
  if (c->sweep_threads && c->sweep_threads != 64 && c->sweep_threads != 128 &&
      c->sweep_threads != 256)
    return fail(MVMC_E_ARG, "sweep_threads must be 0, 64, 128 or 256");
  if (c->exchange_per64 < 0 || c->exchange_per64 > 64)
    return fail(MVMC_E_ARG, "exchange_per64 must be in [0, 64]");
  if (c->exchange_per64 && c->sweep_threads)
    return fail(MVMC_E_ARG, "exchange updates need the register or anti-parallel-block sweep");
  if (c->sweep_variant < 0 || c->sweep_variant > MVMC_N_SWEEP_VARIANTS)
    return fail(MVMC_E_ARG, "sweep_variant must be 0 (automatic) or 1 + a variant");
  if (c->schedule != MVMC_SCHED_BUCKETS && c->schedule != MVMC_SCHED_QUEUE)
    return fail(MVMC_E_ARG, "schedule must be MVMC_SCHED_BUCKETS or MVMC_SCHED_QUEUE");
  if (c->schedule == MVMC_SCHED_QUEUE && c->sweep_threads)
    return fail(MVMC_E_ARG, "the queue schedule takes sweep_threads = 0");
  if (c->schedule == MVMC_SCHED_QUEUE && c->sweep_variant != 0 && c->sweep_variant != 1 &&
      c->sweep_variant != 10)
    return fail(MVMC_E_ARG, "the queue schedule runs variants 0 and 9 only (sweep_variant 0, 1 "
                            "or 10)");
  for (int k = 0; k < c->n_instances; ++k) {
    const mvmc_instance_desc& d = c->inst[k];
    const int ns = d.n_sites;
    if (ns < 3 || ns > kMaxSites) return fail(MVMC_E_SHAPE, "instance %d: n_sites %d outside [3, %d]", k, ns, kMaxSites);
    if (d.n_up < 1 || d.n_dn < 1 || d.n_up > ns || d.n_dn > ns)
      return fail(MVMC_E_SHAPE, "instance %d: electron counts out of range", k);
    if (d.n_up != d.n_dn)
      return fail(MVMC_E_SHAPE, "instance %d: anti-parallel pairing needs n_up == n_dn", k);
    if (d.n_up + d.n_dn > kMaxElec) return fail(MVMC_E_SHAPE, "instance %d: too many electrons", k);
    if (d.n_walkers < 1) return fail(MVMC_E_SHAPE, "instance %d: n_walkers < 1", k);
    if (d.n_bonds < 0 || (d.n_bonds > 0 && (!d.bond_i || !d.bond_j || !d.bond_t)))
      return fail(MVMC_E_ARG, "instance %d: bond arrays missing", k);
    for (int b = 0; b < d.n_bonds; ++b) {
      if (d.bond_i[b] < 0 || d.bond_i[b] >= ns || d.bond_j[b] < 0 || d.bond_j[b] >= ns ||
          d.bond_i[b] == d.bond_j[b])
        return fail(MVMC_E_ARG, "instance %d: bond %d out of range", k, b);
      if (!std::isfinite(d.bond_t[b])) return fail(MVMC_E_NONFINITE, "instance %d: bond_t not finite", k);
    }
    if (!d.U || !d.f_idx || !d.g_idx || !d.v_idx) return fail(MVMC_E_ARG, "instance %d: map missing", k);
    for (int i = 0; i < ns; ++i)
      if (!std::isfinite(d.U[i])) return fail(MVMC_E_NONFINITE, "instance %d: U not finite", k);
    if (d.n_f < 0 || d.n_g < 0 || d.n_v < 0 || d.n_hidden < 0)
      return fail(MVMC_E_ARG, "instance %d: negative parameter count", k);
    for (int e = 0; e < ns * ns; ++e) {
      if (d.f_idx[e] < -1 || d.f_idx[e] >= d.n_f) return fail(MVMC_E_ARG, "instance %d: f_idx[%d] out of range", k, e);
      if (d.v_idx[e] < -1 || d.v_idx[e] >= d.n_v) return fail(MVMC_E_ARG, "instance %d: v_idx[%d] out of range", k, e);
      const int i = e / ns, j = e % ns;
      if (d.v_idx[e] != d.v_idx[j * ns + i]) return fail(MVMC_E_ARG, "instance %d: v_idx not symmetric", k);
      if (i == j && d.v_idx[e] != -1) return fail(MVMC_E_ARG, "instance %d: v_idx diagonal must be -1", k);
    }
    for (int i = 0; i < ns; ++i)
      if (d.g_idx[i] < -1 || d.g_idx[i] >= d.n_g) return fail(MVMC_E_ARG, "instance %d: g_idx out of range", k);
    if (d.n_proj < 0 || d.n_proj > MVMC_MAX_PROJ)
      return fail(MVMC_E_ARG, "instance %d: n_proj %d outside [0, %d]", k, d.n_proj, MVMC_MAX_PROJ);
    if (d.n_proj > 0) {
      if (!d.proj_map || !d.proj_weight)
        return fail(MVMC_E_ARG, "instance %d: projection maps or weights missing", k);
      bool any_w = false;
      for (int p = 0; p < d.n_proj; ++p) {
        if (!std::isfinite(d.proj_weight[p]))
          return fail(MVMC_E_NONFINITE, "instance %d: projection weight %d not finite", k, p);
        any_w = any_w || d.proj_weight[p] != 0.0;
        std::vector<char> seen(ns, 0);
        for (int i = 0; i < ns; ++i) {
          const int32_t t = d.proj_map[(size_t)p * ns + i];
          if (t < 0 || t >= ns || seen[t])
            return fail(MVMC_E_ARG, "instance %d: projection map %d is not a permutation", k, p);
          seen[t] = 1;
        }
      }
      if (!any_w) return fail(MVMC_E_ARG, "instance %d: every projection weight is zero", k);
      if (c->exchange_per64)
        return fail(MVMC_E_ARG, "instance %d: projected states take hopping updates only "
                                "(exchange_per64 = 0)", k);
      if (c->schedule == MVMC_SCHED_QUEUE)
        return fail(MVMC_E_ARG, "instance %d: projected states need MVMC_SCHED_BUCKETS", k);
    }
  }
  return Err{};
}

int64_t nparams_of(const mvmc_instance_desc& d) {
  const int64_t n2 = 2 * (int64_t)d.n_sites;
  const int64_t rbm = d.n_hidden ? n2 + d.n_hidden + (int64_t)d.n_hidden * n2 : 0;
  return (int64_t)d.n_f + d.n_g + d.n_v + rbm;
}

int64_t f_members(const mvmc_instance_desc& d) {
  int64_t m = 0;
  for (int e = 0; e < d.n_sites * d.n_sites; ++e) m += d.f_idx[e] >= 0;
  return m;
}
int64_t v_members(const mvmc_instance_desc& d) {
  int64_t m = 0;
  const int ns = d.n_sites;
  for (int i = 0; i < ns; ++i)
    for (int j = i + 1; j < ns; ++j) m += d.v_idx[i * ns + j] >= 0;
  return m;
}

// Sweep variant of instance k: 0 register tier, 1-3 LDS kernel with
// 64/128/256 threads, 4-6 HBM kernel with 64/128/256 threads (both keep the
// full X^-1), 7-9 anti-parallel-block kernel (M^-1 alone in LDS) with
// 64/128/256 threads.  Exchange updates run on 0 and 7-9 only.
bool variant_fits(const Plan& P, int k, int v) {
  const InstDev& I = P.inst[k];
  if (I.nproj) return false;   // projected instances have a sweep of their own
  if (P.exchange && v >= 1 && v <= 6) return false;
  if (P.queue) {
    if (v != 0 && v != 9) return false;
    // the anti-parallel walkers refresh by the 16 x 16 tile inside the launch
    if (v == 9 && (sweep_queue_nb(I.ne) <= 0 ||
                   sweep_queue_lds_bytes(0, I.ne, I.ns, I.M, P.tsize) > kLdsLimit))
      return false;
  }
  if (v == 0) {
    const int rc = sweep_reg_class(I.ne, P.tsize);
    // the queue kernel runs every register-tier group with the 64-electron layout
    return rc && sweep_reg_lds_bytes(P.queue ? 64 : rc, I.ns, I.M, P.tsize, kRegWpb) <= kLdsLimit;
  }
  const int nt = 64 << ((v - 1) % 3);
  if (v >= 7) return sweep_ap_lds_bytes(I.ne, I.ns, I.M, P.tsize, nt) <= kLdsLimit;
  return sweep_lds_bytes(I.ne, I.ns, I.M, v <= 3, P.tsize, nt) <= kLdsLimit;
}
int variant_of(const Plan& P, int k) {
  if (P.inst[k].nproj) return MVMC_N_SWEEP_VARIANTS;
  if (P.reg_class[k]) return 0;
  const int nt = P.sweep_nt[k];
  const int base = P.sweep_ap[k] ? 7 : (P.inst[k].sweep_lds ? 1 : 4);
  return base + (nt == 64 ? 0 : (nt == 128 ? 1 : 2));
}
void set_variant(Plan& P, int k, int v) {
  InstDev& I = P.inst[k];
  if (I.nproj) return;
  if (v == 0) {
    P.reg_class[k] = sweep_reg_class(I.ne, P.tsize);
    P.sweep_ap[k] = 0;
    return;
  }
  P.reg_class[k] = 0;
  P.sweep_nt[k] = 64 << ((v - 1) % 3);
  P.sweep_ap[k] = v >= 7;
  I.sweep_lds = v >= 1 && v <= 3;
}
// Default: the register tier where it fits, else the anti-parallel-block
// kernel (threads by the block side n; one wavefront up to n = 64 in single
// precision, measured at 10 x 10: 9.5 ms against 10.1 ms with two for 10
// sweeps, while double precision prefers two: 11.2 against 12.3 ms), else
// the full-X^-1 kernel from HBM.
int default_variant(const Plan& P, int k) {
  if (variant_fits(P, k, 0)) return 0;
  if (P.queue) return variant_fits(P, k, 9) ? 9 : -1;
  const int n = P.inst[k].ne / 2;
  const int v = 7 + (n <= (P.tsize == 4 ? 64 : 48) ? 0 : (n <= 96 ? 1 : 2));
  if (variant_fits(P, k, v)) return v;
  return P.exchange ? -1 : 6;
}

Plan make_plan(const mvmc_config& c) {
  Plan P;
  P.tsize = c.precision == MVMC_FP64 ? 8 : 4;
  P.exchange = c.exchange_per64 > 0;
  P.queue = c.schedule == MVMC_SCHED_QUEUE;
  const int n = c.n_instances;
  P.inst.resize(n);
  P.sr.resize(n);
  P.reg_class.assign(n, 0);
  P.sweep_nt.assign(n, 256);
  P.sweep_ap.assign(n, 0);
  int64_t off_A = 0, off_V = 0, off_site = 0, off_nptr = 0, off_nbr = 0, off_fm_ptr = 0,
          off_fm = 0, off_gm_ptr = 0, off_gm = 0, off_vm_ptr = 0, off_vm = 0, off_rbm = 0,
          off_Y = 0, off_pos = 0, off_empty = 0, off_h = 0, off_theta = 0, off_chol = 0,
          off_pmap = 0, off_projw = 0, off_pterm = 0,
          off_split = 0, off_colpart = 0, off_syrkpart = 0, off_O = 0, off_S = 0;
  for (int k = 0; k < n; ++k) {
    const mvmc_instance_desc& d = c.inst[k];
    InstDev& I = P.inst[k];
    std::memset(&I, 0, sizeof I);
    I.ns = d.n_sites;
    I.nup = d.n_up;
    I.ndn = d.n_dn;
    I.ne = d.n_up + d.n_dn;
    I.nf = d.n_f;
    I.ng = d.n_g;
    I.nv = d.n_v;
    I.M = d.n_hidden;
    I.W = d.n_walkers;
    I.nproj = d.n_proj;
    I.np = (int32_t)nparams_of(d);
    // O rows padded to 64 parameters, to 128 when the split-bf16 S build
    // takes 128 x 128 tiles (whose operand loads then stay inside the row)
    I.ldO = (int32_t)(wide_params(I.np) ? (I.np + 127) / 128 * 128 : (I.np + 63) / 64 * 64);
    std::vector<int> deg(I.ns, 0);
    for (int b = 0; b < d.n_bonds; ++b) {
      ++deg[d.bond_i[b]];
      ++deg[d.bond_j[b]];
    }
    I.deg_max = 0;
    for (int x : deg) I.deg_max = std::max(I.deg_max, x);
    const int nt = sweep_threads_for(c, I.ne);
    P.sweep_nt[k] = nt;
    I.sweep_lds = sweep_lds_bytes(I.ne, I.ns, I.M, true, P.tsize, nt) <= kLdsLimit;
    if (I.nproj) {   // its own sweep, refresh and measurement kernels
      I.sweep_lds = 0;
      P.any_proj = true;
      const size_t sw = sweep_proj_lds_bytes(I.ne, I.ns, I.M, I.nproj, P.tsize);
      const size_t me = measure_proj_lds_bytes(I.ne, I.ns, I.M, I.nproj);
      P.proj_sweep_lds = std::max(P.proj_sweep_lds, sw);
      P.proj_measure_lds = std::max(P.proj_measure_lds, me);
      if ((sw > kLdsLimit || me > kLdsLimit || refresh_proj_lds_bytes(I.ne, I.ns) > kLdsLimit) &&
          P.bad_variant < 0)
        P.bad_variant = k;
    } else if (c.sweep_variant > 0) {   // forced variant
      if (variant_fits(P, k, c.sweep_variant - 1)) set_variant(P, k, c.sweep_variant - 1);
      else if (P.bad_variant < 0) P.bad_variant = k;
    } else if (c.sweep_threads == 0) {
      const int v = default_variant(P, k);
      if (v >= 0) set_variant(P, k, v);
      else if (P.bad_variant < 0) P.bad_variant = k;
    }
    I.refresh_lds = I.nproj || refresh_lds_bytes(I.ne, I.ns, true) <= kLdsLimit;
    if (!I.refresh_lds) P.need_Y64 = true;
    I.walker_off = P.W;
    I.param_off = P.np;
    I.rows = (int64_t)c.n_slots * I.W;
    I.eloc_off = P.eloc;
    I.O_off = off_O;
    I.S_off = off_S;
    const int64_t n2 = 2 * (int64_t)I.ns;
    I.A_off = off_A;
    off_A += n2 * n2;
    I.V_off = off_V;
    off_V += (int64_t)I.ns * I.ns;
    I.site_off = off_site;
    off_site += I.ns;
    I.nptr_off = off_nptr;
    off_nptr += I.ns + 1;
    I.nbr_off = off_nbr;
    off_nbr += 2 * (int64_t)d.n_bonds;
    I.fm_ptr_off = off_fm_ptr;
    off_fm_ptr += I.nf + 1;
    I.fm_off = off_fm;
    off_fm += f_members(d);
    I.gm_ptr_off = off_gm_ptr;
    off_gm_ptr += I.ng + 1;
    I.gm_off = off_gm;
    off_gm += I.ns;
    I.vm_ptr_off = off_vm_ptr;
    off_vm_ptr += I.nv + 1;
    I.vm_off = off_vm;
    off_vm += v_members(d);
    I.rbm_a_off = off_rbm;
    I.rbm_b_off = off_rbm + (I.M ? n2 : 0);
    I.rbm_W_off = I.rbm_b_off + I.M;
    off_rbm += I.M ? n2 + I.M + I.M * n2 : 0;
    I.Y_off = off_Y;
    I.Y_ld = std::max<int64_t>((int64_t)I.ne * I.ne, (int64_t)I.nproj * I.nup * I.nup);
    off_Y += (int64_t)I.W * I.Y_ld;
    I.proj_off = off_pmap;
    off_pmap += 2 * (int64_t)I.nproj * I.ns;
    I.projw_off = off_projw;
    off_projw += I.nproj;
    I.pterm_off = off_pterm;
    off_pterm += (int64_t)I.W * 2 * I.nproj;
    I.pos_off = off_pos;
    off_pos += (int64_t)I.W * I.ne;
    I.empty_off = off_empty;
    off_empty += (int64_t)I.W * n2;
    I.h_off = off_h;
    off_h += (int64_t)I.W * I.ns;
    I.theta_off = off_theta;
    off_theta += (int64_t)I.W * I.M;
    I.chol_off = off_chol;
    // the factor, then the inverses of its 64 x 64 diagonal blocks
    if (c.build_s && c.solver == MVMC_SOLVE_CHOL)
      off_chol += (int64_t)I.np * I.np + (I.np + 63) / 64 * 64 * 64;
    I.split_off = off_split;
    const int64_t rows32 = (I.rows + 31) / 32 * 32;
    const bool tiled_s = c.build_s && c.precision == MVMC_MIXED && wide_params(I.np);
    const int64_t sld = tiled_s ? split_ld_for(I.np, I.ldO) : I.ldO;
    if (c.build_s && c.precision == MVMC_MIXED) off_split += 2 * rows32 * sld;

    SrInst& S = P.sr[k];
    std::memset(&S, 0, sizeof S);
    S.np = I.np;
    S.ldO = I.ldO;
    S.rows = I.rows;
    S.walkers = I.W;
    S.O_off = I.O_off;
    S.S_off = I.S_off;
    S.eloc_off = I.eloc_off;
    S.param_off = I.param_off;
    S.chol_off = I.chol_off;
    S.split_off = I.split_off;
    S.split_rows = rows32;
    S.split_ld = sld;
    S.colpart_off = off_colpart;
    off_colpart += 3 * ((I.rows + kRowChunk - 1) / kRowChunk) * I.ldO;
    const int64_t ntile = (I.np + 63) / 64;
    const int64_t tiles = ntile * (ntile + 1) / 2;
    int64_t ks = std::max<int64_t>(1, 1024 / std::max<int64_t>(tiles, 1));
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, I.rows / 256));
    while (ks > 1 && ks * tiles * 4096 * 8 > ((int64_t)256 << 20)) ks /= 2;
    // wide parameter sets: direct-to-LDS tiles (256 by default), no sample
    // split except for the tail tiles, whose FP32 partials share this pool;
    // in double precision 128 x 128 tiles written straight into S
    S.wide64 = c.build_s && c.precision == MVMC_FP64 && wide_params(I.np);
    if (tiled_s || S.wide64) ks = 1;
    S.ksplit = (int32_t)ks;
    S.sb = tiled_s ? kMaxTileSb : 0;
    S.syrkpart_off = off_syrkpart;
    if (c.build_s && !S.wide64)
      off_syrkpart += tiled_s ? (int64_t)kTailUnitsMax * (64 * kMaxTileSb) * (64 * kMaxTileSb) / 2
                              : ks * tiles * 4096;
    else if (S.wide64)
      off_syrkpart += (int64_t)kWideTailUnits * kWideTile * kWideTile;

    off_O += I.rows * I.ldO;
    if (c.build_s) off_S += (int64_t)I.np * I.np;
    P.W += I.W;
    P.np += I.np;
    P.eloc += I.rows;
    P.Y_elems += (int64_t)I.W * I.Y_ld;
    P.max_ne = std::max(P.max_ne, I.ne);
    P.max_ns = std::max(P.max_ns, I.ns);
    P.max_M = std::max(P.max_M, I.M);
    P.max_np = std::max<int64_t>(P.max_np, I.np);
    P.max_ld = std::max<int64_t>(P.max_ld, I.ldO);
    P.max_sld = std::max<int64_t>(P.max_sld, S.split_ld);
    P.max_rows = std::max<int64_t>(P.max_rows, I.rows);
    P.max_ksplit = std::max<int>(P.max_ksplit, S.ksplit);
  }
  P.O_elems = off_O;
  P.S_elems = c.build_s ? off_S : 0;

  size_t cur = 0;
  auto take = [&](Pool& p, size_t bytes) {
    p.off = cur;
    p.bytes = bytes;
    cur = align_up(cur + std::max<size_t>(bytes, 1));
  };
  const size_t W = (size_t)P.W;
  take(P.inst_p, sizeof(InstDev) * n);
  take(P.srinst_p, sizeof(SrInst) * n);
  take(P.walker_inst, 4 * W);
  // [sweep lists or queue groups and items | refresh lists | all walkers |
  //  scratch | queue head]
  take(P.lists, 4 * (6 * W + 2 * (size_t)kRegWpb * n) + 64);
  take(P.A64, 8 * (size_t)off_A);
  take(P.A32, 4 * (size_t)off_A);
  take(P.V, 8 * (size_t)off_V);
  take(P.fidx, 4 * (size_t)off_V);
  take(P.vidx, 4 * (size_t)off_V);
  take(P.G, 8 * (size_t)off_site);
  take(P.U, 8 * (size_t)off_site);
  take(P.gidx, 4 * (size_t)off_site);
  take(P.nbr_ptr, 4 * (size_t)off_nptr);
  take(P.nbr_site, 4 * (size_t)off_nbr);
  take(P.nbr_t, 8 * (size_t)off_nbr);
  take(P.fm_ptr, 4 * (size_t)off_fm_ptr);
  take(P.fm, 4 * (size_t)off_fm);
  take(P.gm_ptr, 4 * (size_t)off_gm_ptr);
  take(P.gm, 4 * (size_t)off_gm);
  take(P.vm_ptr, 4 * (size_t)off_vm_ptr);
  take(P.vm, 4 * (size_t)off_vm);
  take(P.rbm64, 8 * (size_t)off_rbm);
  take(P.rbm32, 4 * (size_t)off_rbm);
  take(P.rbmT64, 8 * (size_t)off_rbm);
  take(P.rbmT32, 4 * (size_t)off_rbm);
  take(P.Y, P.tsize * (size_t)off_Y);
  take(P.Y64, P.need_Y64 ? 8 * (size_t)off_Y : 0);
  take(P.pos, 4 * (size_t)off_pos);
  take(P.empty, 4 * (size_t)off_empty);
  take(P.h, 8 * (size_t)off_h);
  take(P.theta, 8 * (size_t)off_theta);
  take(P.pmap, 4 * (size_t)off_pmap);
  take(P.projw, 8 * (size_t)off_projw);
  take(P.pterm, 8 * (size_t)off_pterm);
  take(P.cnt, 8 * W);
  take(P.upd, 8 * W);
  take(P.target, 8 * W);
  take(P.needs_refresh, 4 * W);
  take(P.accepted, 8 * W);
  take(P.logpf, 8 * W);
  take(P.sgnpf, 8 * W);
  take(P.minpiv, 8 * W);
  take(P.status, 4 * W);
  take(P.guard, 4 * W);
  take(P.chk, 8);
  take(P.lz, 7 * 8 * (size_t)n);
  take(P.trace_base, 8 * W);
  const size_t NP = (size_t)P.np;
  take(P.obar, 8 * NP);
  take(P.sdiag, 8 * NP);
  take(P.x, 8 * NP);
  take(P.r, 8 * NP);
  take(P.p, 8 * NP);
  take(P.w, 8 * NP);
  take(P.shift, 8 * NP);
  take(P.mask, 8 * NP);
  take(P.dotpart, 8 * (size_t)kDotParts * n);
  take(P.t, 8 * (size_t)P.eloc);
  take(P.scal, 8 * (size_t)kScal * n);
  take(P.colpart, 8 * (size_t)off_colpart);
  take(P.syrkpart, 8 * (size_t)off_syrkpart);
  take(P.chol, 8 * (size_t)off_chol);
  take(P.split, 2 * (size_t)off_split);
  P.total = cur;
  return P;
}

HostInst host_tables(const mvmc_instance_desc& d) {
  HostInst H;
  const int ns = d.n_sites;
  H.f_idx.assign(d.f_idx, d.f_idx + ns * ns);
  H.v_idx.assign(d.v_idx, d.v_idx + ns * ns);
  H.g_idx.assign(d.g_idx, d.g_idx + ns);
  H.U.assign(d.U, d.U + ns);
  std::vector<std::vector<std::pair<int, double>>> nb(ns);
  for (int b = 0; b < d.n_bonds; ++b) {
    nb[d.bond_i[b]].push_back({d.bond_j[b], d.bond_t[b]});
    nb[d.bond_j[b]].push_back({d.bond_i[b], d.bond_t[b]});
  }
  H.nbr_ptr.push_back(0);
  for (int s = 0; s < ns; ++s) {
    for (auto& e : nb[s]) {
      H.nbr_site.push_back(e.first);
      H.nbr_t.push_back(e.second);
    }
    H.nbr_ptr.push_back((int32_t)H.nbr_site.size());
  }
  std::vector<std::vector<int32_t>> fl(d.n_f), gl(d.n_g), vl(d.n_v);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j)
      if (d.f_idx[i * ns + j] >= 0) fl[d.f_idx[i * ns + j]].push_back(i * ns + j);
  for (int i = 0; i < ns; ++i)
    if (d.g_idx[i] >= 0) gl[d.g_idx[i]].push_back(i);
  for (int i = 0; i < ns; ++i)
    for (int j = i + 1; j < ns; ++j)
      if (d.v_idx[i * ns + j] >= 0) vl[d.v_idx[i * ns + j]].push_back(i * ns + j);
  auto csr = [](const std::vector<std::vector<int32_t>>& L, std::vector<int32_t>& ptr,
                std::vector<int32_t>& idx) {
    ptr.push_back(0);
    for (auto& l : L) {
      idx.insert(idx.end(), l.begin(), l.end());
      ptr.push_back((int32_t)idx.size());
    }
  };
  csr(fl, H.fm_ptr, H.fm);
  csr(gl, H.gm_ptr, H.gm);
  csr(vl, H.vm_ptr, H.vm);
  return H;
}

struct Bucket {
  size_t list_off;   // byte offset of its walker list inside the list pool
  int n = 0, max_ne = 0, max_ns = 0, max_M = 0, nthreads = 256;
  bool lds = true;
  int reg = 0;       // register-sweep tier (n = number of walker groups) or 0
  bool ap = false;   // anti-parallel-block sweep kernel
  bool proj = false; // projected sweep / refresh kernels
  int inst = -1;     // the one instance of the bucket (autotuning), else -1
};

}  // namespace

// ------------------------------------------------------------------ context
struct mvmc_ctx {
  mvmc_config cfg{};
  std::vector<mvmc_instance_desc> desc;
  Plan plan;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Pools P{};
  SrArgs SA{};
  int32_t* d_all = nullptr;       // every walker, instance order
  int32_t* d_scratch = nullptr;   // redraw list
  std::vector<Bucket> sweep_b, refresh_b;
  // queue schedule: item list (>= 0 anti-parallel walker, < 0 register group
  // -(g + 1)), register groups, queue head; all inside the list pool
  int32_t* q_items = nullptr;
  int32_t* q_groups = nullptr;
  int32_t* q_head = nullptr;
  int q_n = 0, q_ne_reg = 0, q_ne_ap = 0;
  size_t q_lds = 0;                 // largest LDS need of an item
  int32_t* proj_list = nullptr;     // projected walkers (measurement launch)
  int n_proj_walkers = 0;
  std::vector<uint64_t> cnt_host;   // per-instance proposal counter mirror
  TraceRec* trace = nullptr;
  int64_t trace_cap = 0;
  bool sr_ready = false;
  std::string err;
  SrInst* h_sr = nullptr;           // staging of the SR table (pinned unless no_alloc)
  std::vector<SrInst> h_sr_plain;   // its pageable storage for a no-allocation context
  bool no_alloc = false;            // workspace is the static per-device array
  int n_cu = 256;                   // compute units of the device
  bool s_tune = false;              // time the S tile sides at the next mvmc_build_sr
  std::vector<double> s_tile_ms;    // [instance][tile side 128, 192, 256] of the last tuning
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_cat;
  double t_ms[kTimingCats] = {};
  int64_t t_calls[kTimingCats] = {};
};

namespace {

int set_err(mvmc_ctx* c, const Err& e) {
  if (c) c->err = e.msg;
  return e.code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) {                                                                \
      return set_err(ctx, fail(MVMC_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e))); \
    }                                                                                      \
  } while (0)

#define LAUNCHCHK(ctx)                                                                         \
  do {                                                                                         \
    hipError_t _e = hipGetLastError();                                                         \
    if (_e != hipSuccess) return set_err(ctx, fail(MVMC_E_HIP, "kernel launch: %s", hipGetErrorString(_e))); \
  } while (0)

template <typename T>
T* at(char* base, const Pool& p) {
  return reinterpret_cast<T*>(base + p.off);
}

// timing helpers: events bracket a group of launches of one category
int tic(mvmc_ctx* c, int cat) {
  if (!c->timing) return -1;
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1;
    c->ev_pool.push_back({a, b});
    c->ev_cat.push_back(cat);
  }
  const int id = (int)c->ev_used++;
  c->ev_cat[id] = cat;
  (void)hipEventRecord(c->ev_pool[id].first, c->stream);
  return id;
}
void toc(mvmc_ctx* c, int id) {
  if (id >= 0) (void)hipEventRecord(c->ev_pool[id].second, c->stream);
}
void harvest(mvmc_ctx* c) {
  if (!c->ev_used) return;
  (void)hipStreamSynchronize(c->stream);
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[i].first, c->ev_pool[i].second) == hipSuccess) {
      c->t_ms[c->ev_cat[i]] += ms;
      c->t_calls[c->ev_cat[i]] += 1;
    }
  }
  c->ev_used = 0;
}

// Buckets of walkers launched together.  Normally instances that share a
// kernel variant and LDS size class share a bucket; with per_instance (the
// autotuner) every instance gets its own sweep and refresh bucket so that
// its launches can be timed on their own.
void build_buckets(mvmc_ctx* c, bool per_instance = false) {
  const Plan& P = c->plan;
  const int n = c->cfg.n_instances;
  c->sweep_b.clear();
  c->refresh_b.clear();
  // key: (lds flag, LDS size class or 0, threads, instance or -1)
  std::map<std::tuple<int, size_t, int, int>, std::vector<int>> sweep_groups, refresh_groups;
  std::map<std::pair<int, int>, std::vector<int>> reg_groups;
  for (int k = 0; k < n; ++k) {
    const InstDev& I = P.inst[k];
    const int own = per_instance ? k : -1;
    if (I.nproj) {   // projected sweep and refresh (key 3 and 10)
      sweep_groups[{3, 0, 256, own}].push_back(k);
      refresh_groups[{10, 0, 256, own}].push_back(k);
      continue;
    }
    // instances within reach of the anti-parallel block refresh share
    // buckets of their own, so that one large instance does not send the
    // whole bucket to the workgroup-per-walker kernel
    if (const int route = refresh_ap_route(I.ne, I.ns)) {
      refresh_groups[{1 + route, 0, 64, own}].push_back(k);
    } else {
      size_t rb = refresh_lds_bytes(I.ne, I.ns, I.refresh_lds);
      size_t rcls = 4096;
      while (rcls < rb) rcls <<= 1;
      refresh_groups[{I.refresh_lds, rcls, 256, own}].push_back(k);
    }
    if (P.reg_class[k]) {
      reg_groups[{P.reg_class[k], own}].push_back(k);
      continue;
    }
    const int nt = P.sweep_nt[k];
    size_t sb = P.sweep_ap[k] ? sweep_ap_lds_bytes(I.ne, I.ns, I.M, P.tsize, nt)
                              : sweep_lds_bytes(I.ne, I.ns, I.M, I.sweep_lds, P.tsize, nt);
    size_t cls = 4096;
    while (cls < sb) cls <<= 1;
    sweep_groups[{P.sweep_ap[k] ? 2 : (int)I.sweep_lds, cls, nt, own}].push_back(k);
  }
  std::vector<int32_t> lists;
  if (P.queue && !per_instance) {
    // queue schedule: register-tier groups of kRegWpb walkers of one instance
    // (padded with -1), then the items, longest first (cost ~ N_e^2; a group
    // costs as one of its walkers), ties in instance order
    std::vector<std::pair<int64_t, int32_t>> items;
    c->q_ne_reg = c->q_ne_ap = 0;
    c->q_lds = 0;
    for (int k = 0; k < n; ++k) {
      const InstDev& I = P.inst[k];
      const int64_t cost = (int64_t)I.ne * I.ne;
      c->q_lds = std::max(c->q_lds, sweep_queue_lds_bytes(P.reg_class[k] ? I.ne : 0,
                                                          P.reg_class[k] ? 0 : I.ne, I.ns, I.M,
                                                          P.tsize));
      if (P.reg_class[k]) {
        c->q_ne_reg = std::max(c->q_ne_reg, I.ne);
        for (int w = 0; w < I.W; w += kRegWpb) {
          const int32_t g = (int32_t)(lists.size() / kRegWpb);
          for (int u = 0; u < kRegWpb; ++u)
            lists.push_back(w + u < I.W ? (int32_t)(I.walker_off + w + u) : -1);
          items.push_back({cost, -(g + 1)});
        }
      } else {
        c->q_ne_ap = std::max(c->q_ne_ap, I.ne);
        for (int w = 0; w < I.W; ++w) items.push_back({cost, (int32_t)(I.walker_off + w)});
      }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<int64_t, int32_t>& a,
                        const std::pair<int64_t, int32_t>& b) { return a.first > b.first; });
    const size_t items_off = lists.size();
    for (auto& it : items) lists.push_back(it.second);
    c->q_n = (int)items.size();
    char* base = c->ws + P.lists.off;
    c->q_groups = reinterpret_cast<int32_t*>(base);
    c->q_items = reinterpret_cast<int32_t*>(base) + items_off;
  }
  // register tiers: each instance's walkers in groups of kRegWpb, padded with -1
  for (auto& g : reg_groups) {
    if (P.queue && !per_instance) break;
    Bucket b;
    b.reg = g.first.first;
    b.inst = g.first.second;
    b.list_off = lists.size() * 4;
    std::vector<int> ks = g.second;
    std::stable_sort(ks.begin(), ks.end(), [&](int x, int y) { return P.inst[x].ne > P.inst[y].ne; });
    for (int k : ks) {
      const InstDev& I = P.inst[k];
      for (int w = 0; w < I.W; ++w) lists.push_back((int32_t)(I.walker_off + w));
      while ((lists.size() - b.list_off / 4) % kRegWpb) lists.push_back(-1);
      b.max_ne = std::max(b.max_ne, I.ne);
      b.max_ns = std::max(b.max_ns, I.ns);
      b.max_M = std::max(b.max_M, I.M);
    }
    b.n = (int)((lists.size() - b.list_off / 4) / kRegWpb);
    c->sweep_b.push_back(b);
  }
  auto emit = [&](const std::map<std::tuple<int, size_t, int, int>, std::vector<int>>& groups,
                  std::vector<Bucket>& out) {
    for (auto& g : groups) {
      Bucket b;
      b.lds = std::get<0>(g.first) != 0;
      b.ap = &out == &c->sweep_b && std::get<0>(g.first) == 2;
      b.proj = std::get<0>(g.first) == (&out == &c->sweep_b ? 3 : 10);
      b.nthreads = std::get<2>(g.first);
      b.inst = std::get<3>(g.first);
      b.list_off = lists.size() * 4;
      std::vector<int> ks = g.second;
      // longest walkers first (cost ~ N_e^2)
      std::stable_sort(ks.begin(), ks.end(), [&](int a, int bb) {
        return P.inst[a].ne > P.inst[bb].ne;
      });
      for (int k : ks) {
        const InstDev& I = P.inst[k];
        for (int w = 0; w < I.W; ++w) lists.push_back((int32_t)(I.walker_off + w));
        b.max_ne = std::max(b.max_ne, I.ne);
        b.max_ns = std::max(b.max_ns, I.ns);
        b.max_M = std::max(b.max_M, I.M);
      }
      b.n = (int)(lists.size() - b.list_off / 4);
      out.push_back(b);
    }
  };
  if (!(P.queue && !per_instance)) emit(sweep_groups, c->sweep_b);
  emit(refresh_groups, c->refresh_b);
  // projected walkers, for their measurement launch
  const size_t proj_off = lists.size();
  for (int k = 0; k < n; ++k)
    if (P.inst[k].nproj)
      for (int w = 0; w < P.inst[k].W; ++w) lists.push_back((int32_t)(P.inst[k].walker_off + w));
  c->n_proj_walkers = (int)(lists.size() - proj_off);
  c->proj_list = reinterpret_cast<int32_t*>(c->ws + P.lists.off) + proj_off;
  // list pool: [sweep lists (padded) | refresh lists | all walkers | scratch]
  const size_t W = (size_t)P.W;
  std::vector<int32_t> all(W);
  for (size_t w = 0; w < W; ++w) all[w] = (int32_t)w;
  char* base = c->ws + P.lists.off;
  (void)hipMemcpy(base, lists.data(), lists.size() * 4, hipMemcpyHostToDevice);
  c->d_all = reinterpret_cast<int32_t*>(base + lists.size() * 4);
  c->d_scratch = c->d_all + W;
  c->q_head = c->d_scratch + W;
  (void)hipMemcpy(c->d_all, all.data(), W * 4, hipMemcpyHostToDevice);
}

template <typename T>
int refresh_all(mvmc_ctx* c, double sing_tol) {
  const int id = tic(c, 1);
  for (auto& b : c->refresh_b) {
    const int32_t* lst = reinterpret_cast<int32_t*>(c->ws + c->plan.lists.off + b.list_off);
    if (b.proj)
      launch_refresh_proj<T>(c->P, lst, b.n, b.max_ne, b.max_ns, sing_tol, nullptr, c->stream);
    else
      launch_refresh<T>(c->P, lst, b.n, b.max_ne, b.max_ns, b.lds, sing_tol, c->stream);
  }
  toc(c, id);
  LAUNCHCHK(c);
  return MVMC_OK;
}

int refresh_any(mvmc_ctx* c, double sing_tol) {
  return c->cfg.precision == MVMC_FP64 ? refresh_all<double>(c, sing_tol)
                                       : refresh_all<float>(c, sing_tol);
}

// Read walker status; returns the first singular walker or -1.
int first_singular(mvmc_ctx* c, std::vector<int32_t>& st) {
  st.resize(c->plan.W);
  if (hipMemcpyAsync(st.data(), c->P.status, 4 * st.size(), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return -2;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -2;
  for (size_t w = 0; w < st.size(); ++w)
    if (st[w]) return (int)w;
  return -1;
}

// Walkers whose guard word says a ratio stayed non-finite after a double
// refresh: MVMC_E_NONFINITE naming the first one (synchronises the stream).
int check_guard(mvmc_ctx* c) {
  const Plan& P = c->plan;
  std::vector<int32_t> g(P.W);
  std::vector<uint64_t> cnt(P.W);
  HIPCHK(c, hipMemcpyAsync(g.data(), c->P.guard, 4 * P.W, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(cnt.data(), c->P.cnt, 8 * P.W, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->cfg.n_instances; ++k) {
    const InstDev& I = P.inst[k];
    for (int w = 0; w < I.W; ++w)
      if (g[I.walker_off + w] == kGuardFailed)
        return set_err(c, fail(MVMC_E_NONFINITE,
                               "instance %d walker %d (global %lld): ratio of proposal %llu is "
                               "not finite after a double-precision refresh",
                               k, w, (long long)(I.walker_off + w),
                               (unsigned long long)cnt[I.walker_off + w]));
  }
  return MVMC_OK;
}

// MVMC_E_NONFINITE when a parameter vector (device, n doubles) holds a NaN
// or Inf, naming the instance and slot (synchronises the stream).
int check_params(mvmc_ctx* c, const double* d_params, const char* what) {
  const Plan& P = c->plan;
  int64_t* d_first = reinterpret_cast<int64_t*>(c->ws + P.chk.off);
  launch_first_nonfinite(d_params, P.np, d_first, c->stream);
  LAUNCHCHK(c);
  int64_t first = 0;
  HIPCHK(c, hipMemcpyAsync(&first, d_first, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (first >= P.np) return MVMC_OK;
  int k = 0;
  while (k + 1 < c->cfg.n_instances && P.inst[k + 1].param_off <= first) ++k;
  return set_err(c, fail(MVMC_E_NONFINITE, "%s: parameter %lld of instance %d is not finite", what,
                         (long long)(first - P.inst[k].param_off), k));
}

// MVMC_E_SINGULAR naming the first walker whose last refresh found X
// singular (synchronises the stream).
int check_singular(mvmc_ctx* c, const char* when) {
  std::vector<int32_t> st;
  const int bad = first_singular(c, st);
  if (bad == -2) return set_err(c, fail(MVMC_E_HIP, "status read failed"));
  if (bad < 0) return MVMC_OK;
  int k = 0;
  while (k + 1 < c->cfg.n_instances && c->plan.inst[k + 1].walker_off <= bad) ++k;
  return set_err(c, fail(MVMC_E_SINGULAR, "instance %d walker %lld: X is singular %s", k,
                         (long long)(bad - c->plan.inst[k].walker_off), when));
}

int clear_guard(mvmc_ctx* c) {
  HIPCHK(c, hipMemsetAsync(c->P.guard, 0, 4 * c->plan.W, c->stream));
  return MVMC_OK;
}

}  // namespace

// ---------------------------------------------------------------- entry points
extern "C" {

const char* mvmc_status_string(int s) {
  switch (s) {
    case MVMC_OK: return "ok";
    case MVMC_E_ARG: return "invalid argument";
    case MVMC_E_SHAPE: return "inconsistent shape";
    case MVMC_E_WORKSPACE: return "workspace too small or misaligned";
    case MVMC_E_HIP: return "HIP runtime error";
    case MVMC_E_SINGULAR: return "singular matrix";
    case MVMC_E_NONFINITE: return "non-finite value";
    case MVMC_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* mvmc_last_error(const mvmc_ctx* c) { return c ? c->err.c_str() : "no context"; }

int mvmc_query_sizes(const mvmc_config* cfg, mvmc_sizes* out) {
  Err e = validate(cfg);
  if (e.code) return e.code;
  if (!out) return MVMC_E_ARG;
  Plan P = make_plan(*cfg);
  if (P.bad_variant >= 0) return MVMC_E_SHAPE;
  out->n_walkers = P.W;
  out->n_params = P.np;
  out->eloc_elems = P.eloc;
  out->O_elems = P.O_elems;
  out->S_elems = P.S_elems;
  out->Y_elems = P.Y_elems;
  out->pos_elems = (int64_t)(P.pos.bytes / 4);
  out->empty_elems = (int64_t)(P.empty.bytes / 4);
  out->workspace_bytes = (int64_t)P.total;
  out->O_elem_bytes = (int32_t)P.tsize;
  out->pad = 0;
  return MVMC_OK;
}

int mvmc_query_layout(const mvmc_config* cfg, int32_t k, mvmc_instance_layout* out) {
  Err e = validate(cfg);
  if (e.code) return e.code;
  if (!out || k < 0 || k >= cfg->n_instances) return MVMC_E_ARG;
  Plan P = make_plan(*cfg);
  const InstDev& I = P.inst[k];
  out->walker_off = I.walker_off;
  out->n_walkers = I.W;
  out->param_off = I.param_off;
  out->n_params = I.np;
  out->eloc_off = I.eloc_off;
  out->O_off = I.O_off;
  out->O_ld = I.ldO;
  out->S_off = I.S_off;
  out->Y_off = I.Y_off;
  out->pos_off = I.pos_off;
  out->empty_off = I.empty_off;
  out->n_elec = I.ne;
  out->n_sites = I.ns;
  out->Y_ld = I.Y_ld;
  return MVMC_OK;
}

}  // extern "C"

namespace {
int init_impl(mvmc_ctx** out, const mvmc_config* cfg, void* d_ws, size_t ws_bytes,
              const double* d_params, void* hip_stream, bool no_alloc) {
  if (!out) return MVMC_E_ARG;
  *out = nullptr;
  Err e = validate(cfg);
  if (e.code) return e.code;
  if (!d_ws || !d_params) return MVMC_E_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return MVMC_E_WORKSPACE;
  mvmc_ctx* c = new (std::nothrow) mvmc_ctx;
  if (!c) return MVMC_E_ARG;
  c->no_alloc = no_alloc;
  c->cfg = *cfg;
  c->desc.assign(cfg->inst, cfg->inst + cfg->n_instances);
  c->cfg.inst = c->desc.data();
  c->plan = make_plan(c->cfg);
  if (c->plan.bad_variant >= 0) {
    delete c;
    return MVMC_E_SHAPE;
  }
  if (ws_bytes < c->plan.total) {
    delete c;
    return MVMC_E_WORKSPACE;
  }
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char*>(d_ws);
  const Plan& P = c->plan;
  char* b = c->ws;
  Pools& Q = c->P;
  Q.inst = at<InstDev>(b, P.inst_p);
  Q.walker_inst = at<int32_t>(b, P.walker_inst);
  Q.A64 = at<double>(b, P.A64);
  Q.A32 = at<float>(b, P.A32);
  Q.V = at<double>(b, P.V);
  Q.G = at<double>(b, P.G);
  Q.U = at<double>(b, P.U);
  Q.nbr_ptr = at<int32_t>(b, P.nbr_ptr);
  Q.nbr_site = at<int32_t>(b, P.nbr_site);
  Q.nbr_t = at<double>(b, P.nbr_t);
  Q.fidx = at<int32_t>(b, P.fidx);
  Q.vidx = at<int32_t>(b, P.vidx);
  Q.gidx = at<int32_t>(b, P.gidx);
  Q.fm_ptr = at<int32_t>(b, P.fm_ptr);
  Q.fm = at<int32_t>(b, P.fm);
  Q.gm_ptr = at<int32_t>(b, P.gm_ptr);
  Q.gm = at<int32_t>(b, P.gm);
  Q.vm_ptr = at<int32_t>(b, P.vm_ptr);
  Q.vm = at<int32_t>(b, P.vm);
  Q.rbm64 = at<double>(b, P.rbm64);
  Q.rbm32 = at<float>(b, P.rbm32);
  Q.rbmT64 = at<double>(b, P.rbmT64);
  Q.rbmT32 = at<float>(b, P.rbmT32);
  Q.Y = b + P.Y.off;
  Q.Y64 = P.need_Y64 ? at<double>(b, P.Y64) : nullptr;
  Q.pos = at<int32_t>(b, P.pos);
  Q.empty = at<int32_t>(b, P.empty);
  Q.h = at<double>(b, P.h);
  Q.theta = at<double>(b, P.theta);
  Q.cnt = at<uint64_t>(b, P.cnt);
  Q.upd = at<uint64_t>(b, P.upd);
  Q.accepted = at<int64_t>(b, P.accepted);
  Q.logpf = at<double>(b, P.logpf);
  Q.sgnpf = at<double>(b, P.sgnpf);
  Q.minpiv = at<double>(b, P.minpiv);
  Q.status = at<int32_t>(b, P.status);
  Q.guard = at<int32_t>(b, P.guard);
  Q.refresh_upd = c->cfg.refresh_unit == MVMC_REFRESH_UPDATES ? 1 : 0;
  Q.pmap = at<int32_t>(b, P.pmap);
  Q.projw = at<double>(b, P.projw);
  Q.pterm = at<double>(b, P.pterm);
  SrArgs& S = c->SA;
  S.inst = at<SrInst>(b, P.srinst_p);
  S.obar = at<double>(b, P.obar);
  S.sdiag = at<double>(b, P.sdiag);
  S.scal = at<double>(b, P.scal);
  S.colpart = at<double>(b, P.colpart);
  S.syrkpart = at<double>(b, P.syrkpart);
  S.chol = at<double>(b, P.chol);
  S.x = at<double>(b, P.x);
  S.r = at<double>(b, P.r);
  S.p = at<double>(b, P.p);
  S.w = at<double>(b, P.w);
  S.t = at<double>(b, P.t);
  S.shift = at<double>(b, P.shift);
  S.mask = at<double>(b, P.mask);
  S.dotpart = at<double>(b, P.dotpart);

  // static tables
  std::vector<int32_t> winst(P.W);
  std::vector<int32_t> fidx, vidx, gidx, nptr, nsite, fmp, fm, gmp, gm, vmp, vm, pmap;
  std::vector<double> U, nt, projw;
  for (int k = 0; k < cfg->n_instances; ++k) {
    HostInst H = host_tables(c->desc[k]);
    const InstDev& I = P.inst[k];
    for (int w = 0; w < I.W; ++w) winst[I.walker_off + w] = k;
    if (I.nproj) {   // maps q_p, then their inverses
      const mvmc_instance_desc& d = c->desc[k];
      const size_t base = pmap.size();
      pmap.insert(pmap.end(), d.proj_map, d.proj_map + (size_t)I.nproj * I.ns);
      pmap.resize(base + 2 * (size_t)I.nproj * I.ns);
      for (int p = 0; p < I.nproj; ++p)
        for (int i = 0; i < I.ns; ++i)
          pmap[base + (size_t)(I.nproj + p) * I.ns + d.proj_map[(size_t)p * I.ns + i]] = i;
      projw.insert(projw.end(), d.proj_weight, d.proj_weight + I.nproj);
    }
    fidx.insert(fidx.end(), H.f_idx.begin(), H.f_idx.end());
    vidx.insert(vidx.end(), H.v_idx.begin(), H.v_idx.end());
    gidx.insert(gidx.end(), H.g_idx.begin(), H.g_idx.end());
    U.insert(U.end(), H.U.begin(), H.U.end());
    nptr.insert(nptr.end(), H.nbr_ptr.begin(), H.nbr_ptr.end());
    nsite.insert(nsite.end(), H.nbr_site.begin(), H.nbr_site.end());
    nt.insert(nt.end(), H.nbr_t.begin(), H.nbr_t.end());
    fmp.insert(fmp.end(), H.fm_ptr.begin(), H.fm_ptr.end());
    fm.insert(fm.end(), H.fm.begin(), H.fm.end());
    gmp.insert(gmp.end(), H.gm_ptr.begin(), H.gm_ptr.end());
    gm.insert(gm.end(), H.gm.begin(), H.gm.end());
    vmp.insert(vmp.end(), H.vm_ptr.begin(), H.vm_ptr.end());
    vm.insert(vm.end(), H.vm.begin(), H.vm.end());
  }
  auto up = [&](const Pool& p, const void* src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpy(b + p.off, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t he = hipSuccess;
  auto chk = [&](hipError_t x) {
    if (x != hipSuccess && he == hipSuccess) he = x;
  };
  chk(up(P.inst_p, P.inst.data(), sizeof(InstDev) * P.inst.size()));
  chk(up(P.srinst_p, P.sr.data(), sizeof(SrInst) * P.sr.size()));
  chk(up(P.walker_inst, winst.data(), 4 * winst.size()));
  chk(up(P.fidx, fidx.data(), 4 * fidx.size()));
  chk(up(P.vidx, vidx.data(), 4 * vidx.size()));
  chk(up(P.gidx, gidx.data(), 4 * gidx.size()));
  chk(up(P.U, U.data(), 8 * U.size()));
  chk(up(P.nbr_ptr, nptr.data(), 4 * nptr.size()));
  chk(up(P.nbr_site, nsite.data(), 4 * nsite.size()));
  chk(up(P.nbr_t, nt.data(), 8 * nt.size()));
  chk(up(P.fm_ptr, fmp.data(), 4 * fmp.size()));
  chk(up(P.fm, fm.data(), 4 * fm.size()));
  chk(up(P.gm_ptr, gmp.data(), 4 * gmp.size()));
  chk(up(P.gm, gm.data(), 4 * gm.size()));
  chk(up(P.vm_ptr, vmp.data(), 4 * vmp.size()));
  chk(up(P.vm, vm.data(), 4 * vm.size()));
  chk(up(P.pmap, pmap.data(), 4 * pmap.size()));
  chk(up(P.projw, projw.data(), 8 * projw.size()));
  chk(hipMemset(Q.cnt, 0, 8 * P.W));
  chk(hipMemset(Q.upd, 0, 8 * P.W));
  chk(hipMemset(Q.accepted, 0, 8 * P.W));
  chk(hipMemset(Q.guard, 0, 4 * P.W));
  chk(hipMemset(b + P.needs_refresh.off, 0, 4 * P.W));
  chk(hipMemset(Q.theta, 0, 8 * std::max<size_t>(P.theta.bytes / 8, 1)));
  // the same-spin blocks of every X^-1 are zero and only this clear writes them
  chk(hipMemset(Q.Y, 0, std::max<size_t>(P.Y.bytes, 1)));
  chk(hipMemset(S.scal, 0, P.scal.bytes));
  if (c->no_alloc) {
    c->h_sr_plain.resize(P.sr.size());
    c->h_sr = c->h_sr_plain.data();
  } else {
    chk(hipHostMalloc((void**)&c->h_sr, sizeof(SrInst) * P.sr.size(), hipHostMallocDefault));
  }
  if (he != hipSuccess) {
    c->err = std::string("init upload: ") + hipGetErrorString(he);
    mvmc_destroy(c);
    return MVMC_E_HIP;
  }
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu > 0)
      c->n_cu = ncu;
    for (SrInst& S : c->plan.sr) set_tiles(S, S.sb, c->n_cu);
  }
  std::memcpy(c->h_sr, P.sr.data(), sizeof(SrInst) * P.sr.size());
  build_buckets(c);
  c->cnt_host.assign(cfg->n_instances, 0);

  if (int rc = check_params(c, d_params, "init")) {
    std::fprintf(stderr, "mvmc_init_wavefunction: %s\n", c->err.c_str());
    mvmc_destroy(c);
    return rc;
  }
  // parameters -> tables
  launch_expand(Q, P.inst.data(), cfg->n_instances, d_params, c->stream);
  // initial configurations: uniform draws, redrawn while X is singular
  std::vector<int32_t> st;
  std::vector<int32_t> redo(P.W);
  for (int64_t w = 0; w < P.W; ++w) redo[w] = (int32_t)w;
  int attempt = 0;
  for (; attempt < 100 && !redo.empty(); ++attempt) {
    if (hipMemcpy(c->d_scratch, redo.data(), 4 * redo.size(), hipMemcpyHostToDevice) != hipSuccess)
      break;
    launch_draw_configs(Q, c->d_scratch, (int)redo.size(), cfg->seed, (uint32_t)attempt, c->stream);
    launch_build_empty(Q, c->d_scratch, (int)redo.size(), P.max_ns, c->stream);
    int rc = refresh_any(c, 1e-8);
    if (rc) {
      mvmc_destroy(c);
      return rc;
    }
    if (first_singular(c, st) == -2) break;
    redo.clear();
    for (int64_t w = 0; w < P.W; ++w)
      if (st[w]) redo.push_back((int32_t)w);
  }
  if (hipGetLastError() != hipSuccess || !redo.empty()) {
    const int code = redo.empty() ? MVMC_E_HIP : MVMC_E_SINGULAR;
    fprintf(stderr, "mvmc_init_wavefunction: %s (%zu walkers without an invertible start)\n",
            mvmc_status_string(code), redo.size());
    mvmc_destroy(c);
    return code;
  }
  *out = c;
  return MVMC_OK;
}

// The workspace of contexts made by mvmc_init_wavefunction_static: one array
// per device in the code object's device memory.  Host code addresses it
// only through the pointer hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticWorkspaceBytes = MVMC_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

extern "C" {

int mvmc_init_wavefunction(mvmc_ctx** out, const mvmc_config* cfg, void* d_ws, size_t ws_bytes,
                           const double* d_params, void* hip_stream) {
  return init_impl(out, cfg, d_ws, ws_bytes, d_params, hip_stream, false);
}

int mvmc_init_wavefunction_static(mvmc_ctx** out, const mvmc_config* cfg, const double* d_params,
                                  void* hip_stream) {
  if (!out) return MVMC_E_ARG;
  *out = nullptr;
  Err e = validate(cfg);
  if (e.code) return e.code;
  const Plan P = make_plan(*cfg);
  if (P.bad_variant >= 0) return MVMC_E_SHAPE;
  if (P.total > kStaticWorkspaceBytes) {
    std::fprintf(stderr,
                 "mvmc_init_wavefunction_static: the configuration needs %zu bytes of workspace; "
                 "the static workspace holds %zu\n",
                 P.total, kStaticWorkspaceBytes);
    return MVMC_E_WORKSPACE;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MVMC_E_HIP;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (he != hipSuccess || !p) {
        std::fprintf(stderr, "mvmc_init_wavefunction_static: hipGetSymbolAddress: %s\n",
                     hipGetErrorString(he));
        return MVMC_E_HIP;
      }
      g_scratch_ptr[dev] = p;
    }
    ws = g_scratch_ptr[dev];
  }
  return init_impl(out, cfg, ws, kStaticWorkspaceBytes, d_params, hip_stream, true);
}

int mvmc_destroy(mvmc_ctx* c) {
  if (!c) return MVMC_OK;
  for (auto& e : c->ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (c->h_sr && !c->no_alloc) (void)hipHostFree(c->h_sr);
  delete c;
  return MVMC_OK;
}

int mvmc_set_params(mvmc_ctx* c, const double* d_params) {
  if (!c || !d_params) return MVMC_E_ARG;
  if (int rc = check_params(c, d_params, "mvmc_set_params")) return rc;
  launch_expand(c->P, c->plan.inst.data(), c->cfg.n_instances, d_params, c->stream);
  LAUNCHCHK(c);
  if (int rc = clear_guard(c)) return rc;
  if (int rc = refresh_any(c, 0.0)) return rc;
  return check_singular(c, "with the new parameters");
}

int mvmc_refresh(mvmc_ctx* c) {
  if (!c) return MVMC_E_ARG;
  if (int rc = clear_guard(c)) return rc;
  if (int rc = refresh_any(c, 0.0)) return rc;
  return check_singular(c, "at the refresh");
}

}  // extern "C"

namespace {
// Twice the launch cap over R in the update unit: a run then ends mostly at
// a refresh point (a walker makes about R / acceptance proposals between
// them), so few launches end short of one.  At 10 x 10, R = 32, acceptance
// 0.2, 8 R took the mixed sampling from 15.9 ms (cap R) to 12.4 ms per 10
// sweeps; an unbounded cap measured 12.8 ms.
constexpr int kUpdCapX2 = 16;

// The sweeps of one call.  Register-tier walkers refresh inside the sweep
// kernel; LDS-tier walkers stop at every multiple of refresh_every and are
// refreshed between launches.  With inst_ms, every bucket launch is
// bracketed by events and its time added to the bucket's instance (the
// buckets are then per instance).
int run_sweeps(mvmc_ctx* c, int32_t n_sweeps, std::vector<double>* inst_ms) {
  const Plan& P = c->plan;
  const int R = c->cfg.refresh_every;
  if (P.queue && !inst_ms) {
    // one persistent launch: every walker to its target, refreshes inside
    uint64_t* tgt = reinterpret_cast<uint64_t*>(c->ws + P.target.off);
    const uint64_t* tb = reinterpret_cast<uint64_t*>(c->ws + P.trace_base.off);
    launch_set_target(c->P, tgt, P.W, n_sweeps, c->stream);
    LAUNCHCHK(c);
    const bool full = c->trace != nullptr || c->cfg.exchange_per64 > 0 || P.max_M > 0;
    const int id = tic(c, 0);
    const bool ok =
        c->cfg.precision == MVMC_FP64
            ? launch_sweep_queue<double>(c->P, c->q_items, c->q_n, c->q_groups, c->q_head,
                                         c->q_ne_reg, c->q_ne_ap, c->q_lds, full,
                                         c->n_cu, INT32_MAX, c->cfg.seed, c->trace, c->trace_cap,
                                         tb, tgt, R, c->cfg.exchange_per64, c->stream)
            : launch_sweep_queue<float>(c->P, c->q_items, c->q_n, c->q_groups, c->q_head,
                                        c->q_ne_reg, c->q_ne_ap, c->q_lds, full,
                                        c->n_cu, INT32_MAX, c->cfg.seed, c->trace, c->trace_cap,
                                        tb, tgt, R, c->cfg.exchange_per64, c->stream);
    toc(c, id);
    if (!ok) return set_err(c, fail(MVMC_E_SHAPE, "no queue sweep for these shapes"));
    LAUNCHCHK(c);
    for (int k = 0; k < c->cfg.n_instances; ++k)
      c->cnt_host[k] += (uint64_t)n_sweeps * P.inst[k].ne;
    return MVMC_OK;
  }
  // proposals per walker and launch: R, or kUpdCapX2 * R / 2 when R counts
  // applied updates (fewer rounds; a launch's length is then set by its
  // longest run)
  const bool by_upd = c->cfg.refresh_unit == MVMC_REFRESH_UPDATES;
  const int64_t cap = R > 0 ? (by_upd ? std::max<int64_t>(1, (int64_t)R * kUpdCapX2 / 2) : R)
                            : (int64_t)1 << 62;
  int rounds = 1;
  bool lds_refresh = false;
  std::vector<uint64_t> target(c->cfg.n_instances);
  for (int k = 0; k < c->cfg.n_instances; ++k) {
    const uint64_t tot = (uint64_t)n_sweeps * P.inst[k].ne;
    target[k] = tot;
    if (!P.reg_class[k]) {
      lds_refresh = true;
      // enough refresh-aligned rounds for any starting phase (an extra round
      // is an empty launch); independent of the host's view of the counters,
      // so a captured graph stays valid on replay.  Counting applied updates,
      // a launch ends a walker's run at cap proposals (at most tot / cap
      // times) or at a multiple of R updates (at most ceil(tot / R) times).
      if (R > 0) {
        const int64_t per = (tot + R - 1) / R;
        rounds = std::max<int>(
            rounds, (int)(by_upd ? per + (int64_t)tot / cap + 2 : per + 1));
      }
    }
  }
  // one more round for LDS-tier walkers stopped by a non-finite ratio: the
  // refresh between rounds recomputes them and the last launch retries
  if (lds_refresh && n_sweeps > 0) ++rounds;
  uint64_t* tgt = reinterpret_cast<uint64_t*>(c->ws + P.target.off);
  int32_t* nr = reinterpret_cast<int32_t*>(c->ws + P.needs_refresh.off);
  // per-walker end counters on the device: the call enqueues only kernels
  // (graph-capturable) unless the caller asks for a read-back
  launch_set_target(c->P, tgt, P.W, n_sweeps, c->stream);
  LAUNCHCHK(c);
  const uint64_t* tb = reinterpret_cast<uint64_t*>(c->ws + P.trace_base.off);
  std::vector<std::tuple<hipEvent_t, hipEvent_t, int>> ev;
  auto t0 = [&](int inst) -> int {
    if (!inst_ms || inst < 0) return -1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    (void)hipEventRecord(a, c->stream);
    ev.emplace_back(a, b, inst);
    return (int)ev.size() - 1;
  };
  auto t1 = [&](int id) {
    if (id >= 0) (void)hipEventRecord(std::get<1>(ev[id]), c->stream);
  };
  for (int r = 0; r < rounds; ++r) {
    const int id = tic(c, 0);
    for (auto& b : c->sweep_b) {
      const int32_t* lst = reinterpret_cast<int32_t*>(c->ws + P.lists.off + b.list_off);
      if (b.reg) {
        if (r > 0) continue;   // refreshes inside the kernel; done in the first round
        const int cp = INT32_MAX;
        const int e = t0(b.inst);
        const bool ok =
            c->cfg.precision == MVMC_FP64
                ? launch_sweep_reg<double>(c->P, lst, b.n, b.reg, b.max_ns, b.max_M, cp,
                                           c->cfg.seed, c->trace, c->trace_cap, tb, tgt, nr, R,
                                           1, c->cfg.exchange_per64, c->stream)
                : launch_sweep_reg<float>(c->P, lst, b.n, b.reg, b.max_ns, b.max_M, cp,
                                          c->cfg.seed, c->trace, c->trace_cap, tb, tgt, nr, R,
                                          1, c->cfg.exchange_per64, c->stream);
        t1(e);
        if (!ok) return set_err(c, fail(MVMC_E_ARG, "no register sweep tier %d", b.reg));
        continue;
      }
      const int e = t0(b.inst);
      if (b.proj) {
        if (c->cfg.precision == MVMC_FP64)
          launch_sweep_proj<double>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX),
                                    c->cfg.seed, P.proj_sweep_lds, c->trace, c->trace_cap, tb,
                                    tgt, nr, R, c->stream);
        else
          launch_sweep_proj<float>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX),
                                   c->cfg.seed, P.proj_sweep_lds, c->trace, c->trace_cap, tb,
                                   tgt, nr, R, c->stream);
        t1(e);
        continue;
      }
      if (b.ap) {
        if (c->cfg.precision == MVMC_FP64)
          launch_sweep_ap<double>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX),
                                  c->cfg.seed, b.max_ne, b.max_ns, b.max_M, b.nthreads, c->trace,
                                  c->trace_cap, tb, tgt, nr, R, c->cfg.exchange_per64, c->stream);
        else
          launch_sweep_ap<float>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX),
                                 c->cfg.seed, b.max_ne, b.max_ns, b.max_M, b.nthreads, c->trace,
                                 c->trace_cap, tb, tgt, nr, R, c->cfg.exchange_per64, c->stream);
        t1(e);
        continue;
      }
      if (c->cfg.precision == MVMC_FP64)
        launch_sweep<double>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX), c->cfg.seed,
                             b.max_ne, b.max_ns, b.max_M, b.lds, b.nthreads, c->trace,
                             c->trace_cap, tb, tgt, nr, R, c->stream);
      else
        launch_sweep<float>(c->P, lst, b.n, (int)std::min<int64_t>(cap, INT32_MAX), c->cfg.seed,
                            b.max_ne, b.max_ns, b.max_M, b.lds, b.nthreads, c->trace,
                            c->trace_cap, tb, tgt, nr, R, c->stream);
      t1(e);
    }
    toc(c, id);
    LAUNCHCHK(c);
    if (lds_refresh) {
      const int id2 = tic(c, 1);
      for (auto& b : c->refresh_b) {
        // register-tier walkers never ask for this refresh
        if (b.inst >= 0 && P.reg_class[b.inst]) continue;
        const int32_t* lst = reinterpret_cast<int32_t*>(c->ws + P.lists.off + b.list_off);
        const int e = t0(b.inst);
        if (b.proj && c->cfg.precision == MVMC_FP64)
          launch_refresh_proj<double>(c->P, lst, b.n, b.max_ne, b.max_ns, 0.0, nr, c->stream);
        else if (b.proj)
          launch_refresh_proj<float>(c->P, lst, b.n, b.max_ne, b.max_ns, 0.0, nr, c->stream);
        else if (c->cfg.precision == MVMC_FP64)
          launch_refresh_if<double>(c->P, lst, b.n, b.max_ne, b.max_ns, b.lds, nr, c->stream);
        else
          launch_refresh_if<float>(c->P, lst, b.n, b.max_ne, b.max_ns, b.lds, nr, c->stream);
        t1(e);
      }
      toc(c, id2);
      LAUNCHCHK(c);
    }
  }
  for (int k = 0; k < c->cfg.n_instances; ++k) c->cnt_host[k] += target[k];
  if (inst_ms) {
    const hipError_t se = hipStreamSynchronize(c->stream);
    for (auto& e : ev) {
      float ms = 0.f;
      if (se == hipSuccess && hipEventElapsedTime(&ms, std::get<0>(e), std::get<1>(e)) == hipSuccess)
        (*inst_ms)[std::get<2>(e)] += ms;
      (void)hipEventDestroy(std::get<0>(e));
      (void)hipEventDestroy(std::get<1>(e));
    }
    HIPCHK(c, se);
  }
  return MVMC_OK;
}
}  // namespace

extern "C" {

int mvmc_sample_sweeps(mvmc_ctx* c, int32_t n_sweeps, int64_t* h_accepted) {
  if (!c || n_sweeps < 0) return set_err(c, fail(MVMC_E_ARG, "n_sweeps must be >= 0"));
  const Plan& P = c->plan;
  const int rc = run_sweeps(c, n_sweeps, nullptr);
  if (rc) return rc;
  if (h_accepted) {
    std::vector<int64_t> acc(P.W);
    HIPCHK(c, hipMemcpyAsync(acc.data(), c->P.accepted, 8 * P.W, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->cfg.n_instances; ++k) {
      const InstDev& I = P.inst[k];
      int64_t s = 0;
      for (int w = 0; w < I.W; ++w) s += acc[I.walker_off + w];
      h_accepted[k] = s;
    }
    HIPCHK(c, hipMemsetAsync(c->P.accepted, 0, 8 * P.W, c->stream));
    return check_guard(c);
  }
  return MVMC_OK;
}

int mvmc_autotune(mvmc_ctx* c, int32_t n_sweeps, const char* cache_path, double* h_ms) {
  if (!c || n_sweeps < 1) return set_err(c, fail(MVMC_E_ARG, "n_sweeps must be >= 1"));
  if (c->plan.queue)
    return set_err(c, fail(MVMC_E_ARG, "the queue schedule has fixed sweep variants"));
  Plan& P = c->plan;
  const int n = c->cfg.n_instances, nv = MVMC_N_SWEEP_VARIANTS;
  std::vector<double> ms((size_t)n * nv, std::nan(""));
  std::vector<int> chosen(n, -1);
  for (int k = 0; k < n; ++k)   // projected instances keep their own sweep
    if (P.inst[k].nproj) chosen[k] = MVMC_N_SWEEP_VARIANTS;
  // cached choices: "mvmc-sweep precision ne ns M walkers variant" per line
  auto key = [&](int k) {
    const InstDev& I = P.inst[k];
    char buf[128];
    std::snprintf(buf, sizeof buf, "mvmc-sweep %d %d %d %d %d", c->cfg.precision, I.ne, I.ns,
                  I.M, I.W);
    return std::string(buf);
  };
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[256];
      while (std::fgets(line, sizeof line, f)) {
        char tag[32];
        int prec, ne, ns, M, W, v;
        if (std::sscanf(line, "%31s %d %d %d %d %d %d", tag, &prec, &ne, &ns, &M, &W, &v) != 7)
          continue;
        if (std::string(tag) != "mvmc-sweep" || v < 0 || v >= nv) continue;
        for (int k = 0; k < n; ++k) {
          const InstDev& I = P.inst[k];
          if (prec == c->cfg.precision && ne == I.ne && ns == I.ns && M == I.M && W == I.W &&
              !I.nproj && variant_fits(P, k, v))
            chosen[k] = v;
        }
      }
      std::fclose(f);
    }
  }
  std::vector<int> dflt(n);
  for (int k = 0; k < n; ++k) dflt[k] = variant_of(P, k);
  bool any = false;
  for (int k = 0; k < n; ++k) any = any || chosen[k] < 0;
  // one timed call per variant; instances it does not fit (or already
  // chosen) run their default variant untimed
  for (int v = 0; v < nv && any; ++v) {
    std::vector<char> timed(n, 0);
    for (int k = 0; k < n; ++k) {
      const bool t = chosen[k] < 0 && variant_fits(P, k, v);
      set_variant(P, k, t ? v : (chosen[k] >= 0 ? chosen[k] : dflt[k]));
      timed[k] = t;
    }
    build_buckets(c, true);
    std::vector<double> t_inst(n, 0.0);
    const int rc = run_sweeps(c, n_sweeps, &t_inst);
    if (rc) {
      for (int k = 0; k < n; ++k) set_variant(P, k, dflt[k]);
      build_buckets(c);
      return rc;
    }
    for (int k = 0; k < n; ++k)
      if (timed[k]) ms[(size_t)k * nv + v] = t_inst[k];
  }
  FILE* out = cache_path ? std::fopen(cache_path, "a") : nullptr;
  for (int k = 0; k < n; ++k) {
    if (chosen[k] < 0) {
      int best = dflt[k];
      double bm = INFINITY;
      for (int v = 0; v < nv; ++v) {
        const double t = ms[(size_t)k * nv + v];
        if (t == t && t < bm) {
          bm = t;
          best = v;
        }
      }
      chosen[k] = best;
      if (out) std::fprintf(out, "%s %d\n", key(k).c_str(), best);
    }
    set_variant(P, k, chosen[k]);
  }
  if (out) std::fclose(out);
  build_buckets(c);
  c->s_tune = c->cfg.build_s && c->cfg.precision == MVMC_MIXED;
  HIPCHK(c, hipMemsetAsync(c->P.accepted, 0, 8 * P.W, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h_ms) std::memcpy(h_ms, ms.data(), ms.size() * sizeof(double));
  return MVMC_OK;
}

int mvmc_sweep_variants(const mvmc_ctx* c, int32_t* h_variant) {
  if (!c || !h_variant) return MVMC_E_ARG;
  for (int k = 0; k < c->cfg.n_instances; ++k) h_variant[k] = variant_of(c->plan, k);
  return MVMC_OK;
}

int mvmc_s_tiles(const mvmc_ctx* c, int32_t* h_tile, double* h_ms) {
  if (!c || !h_tile) return MVMC_E_ARG;
  const int n = c->cfg.n_instances;
  for (int k = 0; k < n; ++k) h_tile[k] = 64 * c->plan.sr[k].sb;
  if (h_ms)
    for (size_t i = 0; i < (size_t)n * 3; ++i)
      h_ms[i] = i < c->s_tile_ms.size() ? c->s_tile_ms[i] : std::nan("");
  return MVMC_OK;
}

int mvmc_set_s_tile(mvmc_ctx* c, int32_t side) {
  if (!c) return MVMC_E_ARG;
  if (side != 128 && side != 192 && side != 256)
    return set_err(c, fail(MVMC_E_ARG, "S tile side %d is not 128, 192 or 256", side));
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the SR table staging may be in flight
  for (int k = 0; k < c->cfg.n_instances; ++k)
    if (c->plan.sr[k].sb) {
      set_tiles(c->plan.sr[k], side / 64, c->n_cu);
      set_tiles(c->h_sr[k], side / 64, c->n_cu);
    }
  c->s_tune = false;
  return MVMC_OK;
}

namespace {
constexpr int kProbeBlocksMax = 2 * 1024;   // two workgroups per compute unit, up to 1024 CUs
}  // namespace

size_t mvmc_peak_probe_bytes(void) { return sizeof(float) * 256 * (size_t)kProbeBlocksMax; }

int mvmc_peak_probe(int32_t kind, void* d_scratch, void* hip_stream, double* h_tflops) {
  if (kind < 0 || kind > 2 || !d_scratch || !h_tflops) return MVMC_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    return MVMC_E_HIP;
  const int blocks = std::min(2 * ncu, kProbeBlocksMax);
  const int iters = kind == 2 ? 20000 : 2000;
  float* out = reinterpret_cast<float*>(d_scratch);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return MVMC_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return MVMC_E_HIP;
  }
  constexpr int kReps = 3;
  launch_probe(kind, out, blocks, iters, s);   // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < kReps; ++r) launch_probe(kind, out, blocks, iters, s);
  (void)hipEventRecord(e1, s);
  int rc = MVMC_OK;
  float ms = 0.f;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f))
    rc = MVMC_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const double flops = (double)kReps * blocks * 4 * iters * probe_flops_per_wave_iter(kind);
  *h_tflops = flops / (ms * 1e-3) / 1e12;
  return MVMC_OK;
}

int mvmc_measure_energy_and_O(mvmc_ctx* c, int32_t slot, double* d_eloc, void* d_O) {
  if (!c || !d_eloc || !d_O) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  if (slot < 0 || slot >= c->cfg.n_slots)
    return set_err(c, fail(MVMC_E_ARG, "slot %d outside [0, %d)", slot, c->cfg.n_slots));
  const Plan& P = c->plan;
  const int id = tic(c, 2);
  if (c->cfg.precision == MVMC_FP64) {
    launch_measure<double>(c->P, c->d_all, (int)P.W, slot, d_eloc, (double*)d_O, P.max_ne,
                           P.max_ns, P.max_M, c->stream);
    launch_measure_proj<double>(c->P, c->proj_list, c->n_proj_walkers, slot, d_eloc,
                                (double*)d_O, P.proj_measure_lds, c->stream);
  } else {
    launch_measure<float>(c->P, c->d_all, (int)P.W, slot, d_eloc, (float*)d_O, P.max_ne, P.max_ns,
                          P.max_M, c->stream);
    launch_measure_proj<float>(c->P, c->proj_list, c->n_proj_walkers, slot, d_eloc, (float*)d_O,
                               P.proj_measure_lds, c->stream);
  }
  toc(c, id);
  LAUNCHCHK(c);
  return MVMC_OK;
}

int mvmc_measure_h2(mvmc_ctx* c, int32_t slot, double* d_f1, double* d_f2) {
  if (!c || !d_f1 || !d_f2) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  if (slot < 0 || slot >= c->cfg.n_slots)
    return set_err(c, fail(MVMC_E_ARG, "slot %d outside [0, %d)", slot, c->cfg.n_slots));
  const Plan& P = c->plan;
  for (int k = 0; k < c->cfg.n_instances; ++k) {
    const InstDev& I = P.inst[k];
    if (I.M || I.nproj)
      return set_err(c, fail(MVMC_E_ARG, "instance %d: F(x, H^2) covers states without an RBM "
                                         "factor or a quantum-number projection", k));
    if (local_h2_lds_bytes(I.ne, I.ns) > kLdsLimit)
      return set_err(c, fail(MVMC_E_SHAPE, "instance %d: N_s = %d, N_e = %d exceed the LDS of "
                                           "the F(x, H^2) kernel", k, I.ns, I.ne));
  }
  const int id = tic(c, 2);
  if (c->cfg.precision == MVMC_FP64)
    launch_local_h2<double>(c->P, c->d_all, (int)P.W, slot, d_f1, d_f2, P.max_ne, P.max_ns,
                            c->stream);
  else
    launch_local_h2<float>(c->P, c->d_all, (int)P.W, slot, d_f1, d_f2, P.max_ne, P.max_ns,
                           c->stream);
  toc(c, id);
  LAUNCHCHK(c);
  return MVMC_OK;
}

int mvmc_lanczos_first_step(mvmc_ctx* c, int32_t n_used, const double* d_f1, const double* d_f2,
                            double* h_out) {
  if (!c || !d_f1 || !d_f2 || !h_out) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  if (n_used < 1 || n_used > c->cfg.n_slots)
    return set_err(c, fail(MVMC_E_ARG, "n_slots_used %d outside [1, %d]", n_used,
                           c->cfg.n_slots));
  const int n = c->cfg.n_instances;
  double* d_out = reinterpret_cast<double*>(c->ws + c->plan.lz.off);
  launch_lanczos_moments(c->P, n, n_used, d_f1, d_f2, d_out, c->stream);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(h_out, d_out, sizeof(double) * 7 * n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return MVMC_OK;
}

namespace {
// Grid shape of the split-bf16 S build for the current tile choices.
SyrkLaunch syrk_launch(const SrInst* sr, int n) {
  SyrkLaunch L{};
  for (int k = 0; k < n; ++k) {
    const SrInst& S = sr[k];
    if (!S.sb) {
      L.any64 = true;
      continue;
    }
    const int64_t T = 64 * S.sb, nt = (S.np + T - 1) / T, ntl = nt * (nt + 1) / 2;
    const int64_t units = S.nfull + (ntl - S.nfull) * S.tail_ks;
    L.units[S.sb] = std::max<int>(L.units[S.sb], (int)units);
    L.tail[S.sb] = std::max<int>(L.tail[S.sb], (int)(ntl - S.nfull));
  }
  return L;
}

// Times the S build of the wide instances at each direct-to-LDS tile side
// (on the split arrays just written) and keeps the fastest per instance.
// Every instance of a launch takes the same side while it is timed.
int tune_s_tiles(mvmc_ctx* c, const uint16_t* split, float* d_S) {
  const int n = c->cfg.n_instances;
  c->s_tune = false;
  c->s_tile_ms.assign((size_t)n * 3, std::nan(""));
  bool any = false;
  for (int k = 0; k < n; ++k) any = any || c->h_sr[k].sb != 0;
  if (!any) return MVMC_OK;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  std::vector<int> best(n, 0);
  std::vector<double> best_ms(n, INFINITY);
  int rc = MVMC_OK;
  for (int sb = 2; sb <= kMaxTileSb && rc == MVMC_OK; ++sb) {
    for (int k = 0; k < n; ++k)
      if (c->h_sr[k].sb) set_tiles(c->h_sr[k], sb, c->n_cu);
    const SyrkLaunch L = syrk_launch(c->h_sr, n);
    if (hipMemcpyAsync((void*)c->SA.inst, c->h_sr, sizeof(SrInst) * n, hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
      rc = set_err(c, fail(MVMC_E_HIP, "S tile tuning: table upload failed"));
      break;
    }
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {   // the first run warms up
      (void)hipEventRecord(e0, c->stream);
      sr_syrk_bf16x3(c->SA, split, d_S, n, c->plan.max_np, c->plan.max_ksplit, L, c->stream);
      (void)hipEventRecord(e1, c->stream);
      if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = set_err(c, fail(MVMC_E_HIP, "S tile tuning: kernel failed"));
        break;
      }
      (void)hipEventElapsedTime(&ms, e0, e1);
    }
    for (int k = 0; k < n; ++k)
      if (c->h_sr[k].sb) {
        c->s_tile_ms[(size_t)k * 3 + sb - 2] = ms;
        if (ms < best_ms[k]) {
          best_ms[k] = ms;
          best[k] = sb;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int k = 0; k < n; ++k)
    if (c->h_sr[k].sb) {
      set_tiles(c->h_sr[k], best[k] ? best[k] : kMaxTileSb, c->n_cu);
      set_tiles(c->plan.sr[k], c->h_sr[k].sb, c->n_cu);
    }
  if (rc) return rc;
  HIPCHK(c, hipMemcpyAsync((void*)c->SA.inst, c->h_sr, sizeof(SrInst) * n, hipMemcpyHostToDevice,
                           c->stream));
  return MVMC_OK;
}
}  // namespace

int mvmc_build_sr(mvmc_ctx* c, int32_t n_used, const double* d_eloc, void* d_O, void* d_S,
                  double* d_g, double* h_E, double* h_Eerr, double* h_Evar) {
  if (!c || !d_eloc || !d_O || !d_g) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  if (n_used < 1 || n_used > c->cfg.n_slots)
    return set_err(c, fail(MVMC_E_ARG, "n_slots_used %d outside [1, %d]", n_used, c->cfg.n_slots));
  if (d_S && !c->cfg.build_s) return set_err(c, fail(MVMC_E_STATE, "context built with build_s = 0"));
  const Plan& P = c->plan;
  const int n = c->cfg.n_instances;
  HIPCHK(c, hipStreamSynchronize(c->stream));   // staging buffer may still be in flight
  int64_t max_rows = 0;
  for (int k = 0; k < n; ++k) {
    c->h_sr[k].rows = (int64_t)n_used * P.inst[k].W;
    max_rows = std::max(max_rows, c->h_sr[k].rows);
  }
  HIPCHK(c, hipMemcpyAsync((void*)c->SA.inst, c->h_sr, sizeof(SrInst) * n, hipMemcpyHostToDevice,
                           c->stream));
  c->SA.eloc = d_eloc;
  const bool mixed = c->cfg.precision == MVMC_MIXED;
  uint16_t* split = (mixed && d_S) ? reinterpret_cast<uint16_t*>(c->ws + P.split.off) : nullptr;
  int id = tic(c, 3);
  sr_estats(c->SA, n, c->stream);
  if (mixed)
    sr_colstats<float>(c->SA, (float*)d_O, split, d_g, n, std::max(P.max_ld, P.max_sld), max_rows,
                       c->stream);
  else
    sr_colstats<double>(c->SA, (double*)d_O, nullptr, d_g, n, P.max_ld, max_rows, c->stream);
  toc(c, id);
  LAUNCHCHK(c);
  if (d_S) {
    if (mixed && c->s_tune) {
      const int rc = tune_s_tiles(c, split, (float*)d_S);
      if (rc) return rc;
    }
    id = tic(c, 4);
    if (mixed)
      sr_syrk_bf16x3(c->SA, split, (float*)d_S, n, P.max_np, P.max_ksplit,
                     syrk_launch(c->h_sr, n), c->stream);
    else
    {
      bool any_wide = false, any_narrow = false;
      int wide_units = 0, wide_tail = 0;   // launch extents over the wide instances
      for (int k = 0; k < n; ++k) {
        const SrInst& si = c->h_sr[k];
        (si.wide64 ? any_wide : any_narrow) = true;
        if (!si.wide64) continue;
        const int64_t nt = (si.np + kWideTile - 1) / kWideTile, ntl = nt * (nt + 1) / 2;
        wide_units = std::max<int>(wide_units, (int)(si.nfull + (ntl - si.nfull) * si.tail_ks));
        if (si.tail_ks > 1) wide_tail = std::max<int>(wide_tail, (int)(ntl - si.nfull));
      }
      sr_syrk_vec<double, double>(c->SA, (const double*)d_O, (double*)d_S, n, P.max_np,
                                  P.max_ksplit, any_wide, any_narrow, wide_units, wide_tail,
                                  c->stream);
    }
    toc(c, id);
    LAUNCHCHK(c);
  }
  c->sr_ready = true;
  if (h_E || h_Eerr || h_Evar) {
    std::vector<double> sc((size_t)kScal * n);
    HIPCHK(c, hipMemcpyAsync(sc.data(), c->SA.scal, 8 * sc.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) {
      if (h_E) h_E[k] = sc[k * kScal + kEbar];
      if (h_Eerr) h_Eerr[k] = sc[k * kScal + kEerr];
      if (h_Evar) h_Evar[k] = sc[k * kScal + kEvar];
    }
    if (int rc = check_guard(c)) return rc;
    for (int k = 0; k < n; ++k)
      if (!std::isfinite(sc[k * kScal + kEbar]))
        return set_err(c, fail(MVMC_E_NONFINITE, "instance %d: mean local energy is not finite", k));
  }
  return MVMC_OK;
}

int mvmc_sr_update(mvmc_ctx* c, const void* d_S, const void* d_O, const double* d_g, double dtau,
                   double eps_rel, double eps_abs, int32_t solver, double cg_tol, int32_t cg_maxit,
                   double* d_params, double* d_dparams, int32_t* h_cg_iters) {
  if (!c || !d_g || !d_params) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  if (!c->sr_ready) return set_err(c, fail(MVMC_E_STATE, "mvmc_build_sr must run first"));
  if (!std::isfinite(dtau) || !std::isfinite(eps_rel) || !std::isfinite(eps_abs) || eps_rel < 0 ||
      eps_abs < 0)
    return set_err(c, fail(MVMC_E_ARG, "dtau/eps must be finite and eps >= 0"));
  const Plan& P = c->plan;
  const int n = c->cfg.n_instances;
  const bool mixed = c->cfg.precision == MVMC_MIXED;
  const double freeze = 1e-12;
  std::vector<double> sc((size_t)kScal * n);
  if (solver == MVMC_SOLVE_CHOL) {
    if (!d_S || c->cfg.solver != MVMC_SOLVE_CHOL)
      return set_err(c, fail(MVMC_E_STATE, "Cholesky needs d_S and a context built for it"));
    // A rank-deficient S (fewer samples than parameters) built in reduced
    // precision can leave S_reg short of numerical positive definiteness;
    // then the diagonal shift eps_rel is raised tenfold and the
    // factorisation repeated (from S, which it does not overwrite).
    double eps = eps_rel;
    int escalations = 0;
    for (;;) {
      for (int k = 0; k < n; ++k) {
        HIPCHK(c, hipMemsetAsync(c->SA.scal + k * kScal + kFlag, 0, 8, c->stream));
      }
      const int id = tic(c, 5);
      if (mixed)
        sr_cholesky_solve<float>(c->SA, (const float*)d_S, d_g, eps, eps_abs, freeze, n,
                                 P.max_np, c->stream);
      else
        sr_cholesky_solve<double>(c->SA, (const double*)d_S, d_g, eps, eps_abs, freeze, n,
                                  P.max_np, c->stream);
      toc(c, id);
      LAUNCHCHK(c);
      HIPCHK(c, hipMemcpyAsync(sc.data(), c->SA.scal, 8 * sc.size(), hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      int bad = -1;
      for (int k = 0; k < n && bad < 0; ++k)
        if (sc[k * kScal + kFlag] != 0.0) bad = k;
      if (bad < 0) break;
      if (escalations == kMaxShiftEscalations || !(eps > 0))
        return set_err(c, fail(MVMC_E_SINGULAR, "instance %d: S_reg not positive definite "
                                                "(eps_rel raised to %g)", bad, eps));
      eps *= 10.0;
      ++escalations;
    }
    if (h_cg_iters)
      for (int k = 0; k < n; ++k) h_cg_iters[k] = escalations;
  } else if (solver == MVMC_SOLVE_CG) {
    if (!d_O) return set_err(c, fail(MVMC_E_ARG, "CG needs the centred O"));
    if (cg_maxit < 1 || !(cg_tol > 0)) return set_err(c, fail(MVMC_E_ARG, "cg_maxit >= 1 and cg_tol > 0"));
    const int id = tic(c, 5);
    if (mixed)
      sr_cg_begin<float>(c->SA, d_g, eps_rel, eps_abs, freeze, cg_tol, n, P.max_np, c->stream);
    else
      sr_cg_begin<double>(c->SA, d_g, eps_rel, eps_abs, freeze, cg_tol, n, P.max_np, c->stream);
    int64_t max_rows = 0;
    for (int k = 0; k < n; ++k) max_rows = std::max(max_rows, c->h_sr[k].rows);
    for (int it = 1; it <= cg_maxit; ++it) {
      if (mixed)
        sr_cg_iter<float>(c->SA, (const float*)d_O, it, n, P.max_np, max_rows, c->stream);
      else
        sr_cg_iter<double>(c->SA, (const double*)d_O, it, n, P.max_np, max_rows, c->stream);
      if (it % 16 == 0 || it == cg_maxit) {
        LAUNCHCHK(c);
        HIPCHK(c, hipMemcpyAsync(sc.data(), c->SA.scal, 8 * sc.size(), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bool all = true;
        for (int k = 0; k < n; ++k) all = all && sc[k * kScal + kDone] != 0.0;
        if (all) break;
      }
    }
    toc(c, id);
    HIPCHK(c, hipMemcpyAsync(sc.data(), c->SA.scal, 8 * sc.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h_cg_iters)
      for (int k = 0; k < n; ++k) h_cg_iters[k] = (int32_t)sc[k * kScal + kIters];
  } else {
    return set_err(c, fail(MVMC_E_ARG, "unknown solver %d", solver));
  }
  sr_apply(c->SA, dtau, d_params, d_dparams, n, P.max_np, c->stream);
  LAUNCHCHK(c);
  // a non-finite update is reported before it reaches the walkers (the
  // parameter vector then holds it; the walkers keep the previous tables)
  if (int rc = check_params(c, d_params, "mvmc_sr_update")) return rc;
  launch_expand(c->P, P.inst.data(), n, d_params, c->stream);
  LAUNCHCHK(c);
  if (int rc = clear_guard(c)) return rc;
  int rc = refresh_any(c, 0.0);
  if (rc) return rc;
  return check_singular(c, "after the parameter update");
}

int mvmc_get_state(mvmc_ctx* c, int16_t* d_pos, uint64_t* d_counter, int16_t* d_empty) {
  if (!c) return MVMC_E_ARG;
  const Plan& P = c->plan;
  if (d_pos) launch_pos_narrow(c->P.pos, d_pos, (int64_t)(P.pos.bytes / 4), c->stream);
  if (d_empty) launch_pos_narrow(c->P.empty, d_empty, (int64_t)(P.empty.bytes / 4), c->stream);
  LAUNCHCHK(c);
  if (d_counter)
    HIPCHK(c, hipMemcpyAsync(d_counter, c->P.cnt, 8 * P.W, hipMemcpyDeviceToDevice, c->stream));
  return MVMC_OK;
}

int mvmc_set_state(mvmc_ctx* c, const int16_t* d_pos, const uint64_t* d_counter,
                   const int16_t* d_empty) {
  if (!c || !d_pos || !d_counter) return set_err(c, fail(MVMC_E_ARG, "NULL buffer"));
  const Plan& P = c->plan;
  const int64_t npos = (int64_t)(P.pos.bytes / 4), nemp = (int64_t)(P.empty.bytes / 4);
  // validate on the host before touching the walker state
  std::vector<int16_t> pos(npos), emp(d_empty ? nemp : 0);
  std::vector<uint64_t> cnt(P.W);
  HIPCHK(c, hipMemcpyAsync(pos.data(), d_pos, 2 * npos, hipMemcpyDeviceToHost, c->stream));
  if (d_empty)
    HIPCHK(c, hipMemcpyAsync(emp.data(), d_empty, 2 * nemp, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(cnt.data(), d_counter, 8 * P.W, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->cfg.n_instances; ++k) {
    const InstDev& I = P.inst[k];
    for (int w = 0; w < I.W; ++w) {
      if (cnt[I.walker_off + w] != cnt[I.walker_off])
        return set_err(c, fail(MVMC_E_ARG, "instance %d: counters must be equal", k));
      std::vector<char> occ(2 * I.ns, 0);
      const int16_t* p = pos.data() + I.pos_off + (int64_t)w * I.ne;
      for (int a = 0; a < I.ne; ++a) {
        const int lo = a < I.nup ? 0 : I.ns, hi = lo + I.ns;
        if (p[a] < lo || p[a] >= hi || occ[p[a]])
          return set_err(c, fail(MVMC_E_ARG, "instance %d walker %d: bad configuration", k, w));
        occ[p[a]] = 1;
      }
      if (!d_empty) continue;
      // each spin's list: exactly its empty sites, then -1
      for (int sg = 0; sg < 2; ++sg) {
        const int nfree = I.ns - (sg ? I.ndn : I.nup);
        const int16_t* e = emp.data() + I.empty_off + ((int64_t)w * 2 + sg) * I.ns;
        std::vector<char> seen(I.ns, 0);
        for (int j = 0; j < I.ns; ++j) {
          const int site = e[j];
          const bool ok = j < nfree ? (site >= 0 && site < I.ns && !occ[site + sg * I.ns] &&
                                       !seen[site])
                                    : site == -1;
          if (!ok)
            return set_err(c, fail(MVMC_E_ARG, "instance %d walker %d: bad empty-site list", k,
                                   w));
          if (j < nfree) seen[site] = 1;
        }
      }
    }
  }
  launch_pos_widen(d_pos, c->P.pos, npos, c->stream);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(c->P.cnt, d_counter, 8 * P.W, hipMemcpyDeviceToDevice, c->stream));
  // the count of applied updates restarts with the loaded state (refresh
  // points in the update unit then follow from the state alone)
  HIPCHK(c, hipMemsetAsync(c->P.upd, 0, 8 * P.W, c->stream));
  if (d_empty)
    launch_pos_widen(d_empty, c->P.empty, nemp, c->stream);
  else
    launch_build_empty(c->P, c->d_all, (int)P.W, P.max_ns, c->stream);
  LAUNCHCHK(c);
  for (int k = 0; k < c->cfg.n_instances; ++k) c->cnt_host[k] = cnt[P.inst[k].walker_off];
  if (int r0 = clear_guard(c)) return r0;
  int rc = refresh_any(c, 0.0);
  if (rc) return rc;
  return check_singular(c, "for the loaded configuration");
}

int mvmc_get_inverse(mvmc_ctx* c, double* d_Y) {
  if (!c || !d_Y) return MVMC_E_ARG;
  const Plan& P = c->plan;
  if (c->cfg.precision == MVMC_FP64) {
    HIPCHK(c, hipMemcpyAsync(d_Y, c->P.Y, 8 * P.Y_elems, hipMemcpyDeviceToDevice, c->stream));
  } else {
    launch_widen(reinterpret_cast<const float*>(c->P.Y), d_Y, P.Y_elems, c->stream);
    LAUNCHCHK(c);
  }
  return MVMC_OK;
}

int mvmc_get_pfaffian(mvmc_ctx* c, double* d_logabs, double* d_sign) {
  if (!c) return MVMC_E_ARG;
  if (d_logabs)
    HIPCHK(c, hipMemcpyAsync(d_logabs, c->P.logpf, 8 * c->plan.W, hipMemcpyDeviceToDevice, c->stream));
  if (d_sign)
    HIPCHK(c, hipMemcpyAsync(d_sign, c->P.sgnpf, 8 * c->plan.W, hipMemcpyDeviceToDevice, c->stream));
  return MVMC_OK;
}

int mvmc_trace_enable(mvmc_ctx* c, void* d_trace, int64_t cap) {
  if (!c || cap < 0) return MVMC_E_ARG;
  if (!d_trace || cap == 0) {
    c->trace = nullptr;
    c->trace_cap = 0;
    return MVMC_OK;
  }
  HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.trace_base.off, c->P.cnt, 8 * c->plan.W,
                           hipMemcpyDeviceToDevice, c->stream));
  c->trace = reinterpret_cast<TraceRec*>(d_trace);
  c->trace_cap = cap;
  return MVMC_OK;
}

int mvmc_timing(mvmc_ctx* c, int32_t enable, double* h_ms, int64_t* h_calls) {
  if (!c) return MVMC_E_ARG;
  harvest(c);
  if (h_ms)
    for (int i = 0; i < kTimingCats; ++i) h_ms[i] = c->t_ms[i];
  if (h_calls)
    for (int i = 0; i < kTimingCats; ++i) h_calls[i] = c->t_calls[i];
  if (enable && !c->timing)
    for (int i = 0; i < kTimingCats; ++i) {
      c->t_ms[i] = 0.0;
      c->t_calls[i] = 0;
    }
  c->timing = enable != 0;
  return MVMC_OK;
}

}  // extern "C"
