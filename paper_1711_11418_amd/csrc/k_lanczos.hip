// First-step power-Lanczos (section 3.4): the local values F(x, H) and
// F(x, H^2) = <x|H^2|psi>/<x|psi> of one sample slot, then the moments
// h1, h2(11), h2(20), h3(12), the optimal alpha_1 and E_1(alpha_1).
//
// F(x, H^2) sums every two-step path x -> x' -> x'' of the Hamiltonian:
//   F(x, H^2) = E_U(x) F(x, H) + sum over hops x -> x' of
//               (-t) [ E_U(x') R(x') + sum over hops x' -> x'' of (-t) R(x'') ]
// with R(y) = psi(y)/psi(x) and E_U the on-site energy.  Every end point is
// at most two electron moves away from x, so all Pfaffian ratios follow from
// M^-1 (the anti-parallel block, Eq. AP-Pf: X = [[0, M], [-M^T, 0]],
// M[i][b] = f(site of up i, site of down b), W = M^-1 indexed [b][i]) and
// three products formed once per walker:
//   P[r][i] = sum_b f(r, s_b) W[b][i]        (N_s x n)
//   Q[b][q] = sum_i W[b][i] f(s_i, q)        (n x N_s)
//   T[r][q] = sum_i P[r][i] f(s_i, q)        (N_s x N_s)
// by the matrix-determinant lemma for one or two changed rows/columns of M:
//   up i -> r                      P[r][i]
//   down b -> q                    Q[b][q]
//   up i -> r and up j -> r2       P[r][i] P[r2][j] - P[r2][i] P[r][j]
//   down b -> q and down c -> q2   Q[b][q] Q[c][q2] - Q[b][q2] Q[c][q]
//   up i -> r and down b -> q      P[r][i] Q[b][q] - W[b][i] (T[r][q] - f(r, q))
// (the last is the rank-2 lemma with row i and column b replaced; the
// corner term f(r, q) is the pair of both new sites).  The Gutzwiller and
// Jastrow factors of a double move are taken one move after the other: the
// Jastrow field after moving charge i -> j is h'_l = h_l + v_lj - v_li.
// One workgroup per walker keeps W, P, Q and T in LDS in double; thread t
// takes first moves t, t + 256, ... and sums all second moves from each.
#include "launch.h"

namespace mvmc {

namespace {
constexpr int kH2Threads = 256;

__host__ __device__ inline size_t h2a(size_t x) { return (x + 15) & ~(size_t)15; }

struct H2Lds {
  size_t W, P, Q, T, h, red, ints, total;
  int ldw, ldp, ldq, ldt;
};
// Odd row strides spread the column reads of the products over the banks.
__host__ __device__ inline H2Lds h2_layout(int ne, int ns) {
  H2Lds L;
  const int n = ne / 2;
  L.ldw = n | 1;
  L.ldp = n | 1;
  L.ldq = ns | 1;
  L.ldt = ns | 1;
  L.W = h2a((size_t)n * L.ldw * sizeof(double));
  L.P = h2a((size_t)ns * L.ldp * sizeof(double));
  L.Q = h2a((size_t)n * L.ldq * sizeof(double));
  L.T = h2a((size_t)ns * L.ldt * sizeof(double));
  L.h = h2a((size_t)ns * sizeof(double));
  L.red = h2a(16 * sizeof(double));
  L.ints = h2a((size_t)(ne + 2 * ns) * sizeof(int32_t));
  L.total = L.W + L.P + L.Q + L.T + L.h + L.red + L.ints;
  return L;
}

template <typename T>
__global__ __launch_bounds__(kH2Threads) void k_local_h2(Pools P, const int32_t* __restrict__ wlist,
                                                         int slot, double* __restrict__ f1_out,
                                                         double* __restrict__ f2_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = wlist[blockIdx.x];
  const InstDev& I = P.inst[P.walker_inst[gw]];
  const int ne = I.ne, ns = I.ns, n2 = 2 * ns, n = I.nup;
  const int64_t lw = gw - I.walker_off;
  const int tid = threadIdx.x;
  const H2Lds L = h2_layout(ne, ns);
  unsigned char* q = smem;
  double* Ws = (double*)q;  q += L.W;     // W[b][i] = M^-1
  double* Ps = (double*)q;  q += L.P;     // P[r][i]
  double* Qs = (double*)q;  q += L.Q;     // Q[b][q]
  double* Ts = (double*)q;  q += L.T;     // T[r][q]
  double* hs = (double*)q;  q += L.h;     // Jastrow field
  double* red = (double*)q; q += L.red;
  int32_t* pos = (int32_t*)q;             // ne spin-orbitals
  int32_t* eidx = pos + ne;               // 2 ns: electron at spin-orbital or -1

  const T* Yg = (const T*)P.Y + I.Y_off + lw * ne * ne;
  const int32_t* posg = P.pos + I.pos_off + lw * ne;
  for (int v = tid; v < n2; v += kH2Threads) eidx[v] = -1;
  for (int l = tid; l < ns; l += kH2Threads) hs[l] = P.h[I.h_off + lw * ns + l];
  // W[b][i] = X^-1[n + b][i] (lower-left block)
  for (int e = tid; e < n * n; e += kH2Threads) {
    const int b = e / n, i = e - (e / n) * n;
    Ws[b * L.ldw + i] = (double)Yg[(int64_t)(n + b) * ne + i];
  }
  __syncthreads();
  for (int b = tid; b < ne; b += kH2Threads) {
    pos[b] = posg[b];
    eidx[posg[b]] = b;
  }
  __syncthreads();

  const double* A = P.A64 + I.A_off;
  // pair amplitude f(i, j) = A[(i, up)][(j, dn)]
  auto f = [&](int i, int j) -> double { return A[(int64_t)i * n2 + ns + j]; };
  for (int e = tid; e < ns * n; e += kH2Threads) {
    const int r = e / n, i = e - (e / n) * n;
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += f(r, pos[n + b] - ns) * Ws[b * L.ldw + i];
    Ps[r * L.ldp + i] = s;
  }
  for (int e = tid; e < n * ns; e += kH2Threads) {
    const int b = e / ns, qq = e - (e / ns) * ns;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += Ws[b * L.ldw + i] * f(pos[i], qq);
    Qs[b * L.ldq + qq] = s;
  }
  __syncthreads();
  for (int e = tid; e < ns * ns; e += kH2Threads) {
    const int r = e / ns, qq = e - (e / ns) * ns;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += Ps[r * L.ldp + i] * f(pos[i], qq);
    Ts[r * L.ldt + qq] = s;
  }
  __syncthreads();

  const double* V = P.V + I.V_off;
  const double* G = P.G + I.site_off;
  const double* Uv = P.U + I.site_off;
  const int32_t* nptr = P.nbr_ptr + I.nptr_off;
  const int32_t* nsite = P.nbr_site + I.nbr_off;
  const double* nt = P.nbr_t + I.nbr_off;
  auto occ = [&](int site, int spin) -> int { return eidx[site + spin * ns] >= 0 ? 1 : 0; };

  // on-site energy of x (every thread forms the same sum)
  double eu = 0.0;
  for (int i = 0; i < ns; ++i) eu += (occ(i, 0) && occ(i, 1)) ? Uv[i] : 0.0;

  double e_part = 0.0, f2_part = 0.0;
  const int deg = I.deg_max;
  for (int t1 = tid; t1 < ne * deg; t1 += kH2Threads) {
    const int a = t1 / deg, k1 = t1 - (t1 / deg) * deg;
    const int sa = a >= n ? 1 : 0;
    const int si = pos[a] - sa * ns;                 // site i of electron a
    const int nb1 = nptr[si] + k1;
    if (nb1 >= nptr[si + 1]) continue;
    const int sj = nsite[nb1];                       // site j
    if (occ(sj, sa)) continue;
    const int op = 1 - sa;
    // first move a: i -> j
    const double pf1 = sa == 0 ? Ps[sj * L.ldp + a] : Qs[(a - n) * L.ldq + sj];
    const double lc1 = G[sj] * occ(sj, op) - G[si] * occ(si, op) + hs[sj] - hs[si] -
                       V[(int64_t)si * ns + sj];
    const double r1 = pf1 * exp(lc1);
    const double t1amp = -nt[nb1];
    e_part += t1amp * r1;
    // occupation after the first move
    auto occ1 = [&](int site, int spin) -> int {
      if (spin != sa) return occ(site, spin);
      if (site == sj) return 1;
      if (site == si) return 0;
      return occ(site, spin);
    };
    const double eu1 = eu + (occ(sj, op) ? Uv[sj] : 0.0) - (occ(si, op) ? Uv[si] : 0.0);
    double s2 = eu1 * r1;
    for (int c = 0; c < ne; ++c) {
      const int sc = c >= n ? 1 : 0;
      const int cs = c == a ? sj : pos[c] - sc * ns;   // site of c in x'
      const int oc = 1 - sc;
      for (int nb2 = nptr[cs]; nb2 < nptr[cs + 1]; ++nb2) {
        const int sk = nsite[nb2];
        if (occ1(sk, sc)) continue;
        double r2;
        if (c == a && sk == si) {
          r2 = 1.0;                                    // back to x
        } else {
          double pf2;
          if (c == a) {                                // a: i -> k in one move
            pf2 = sa == 0 ? Ps[sk * L.ldp + a] : Qs[(a - n) * L.ldq + sk];
          } else if (sc == sa) {
            if (sa == 0)
              pf2 = Ps[sj * L.ldp + a] * Ps[sk * L.ldp + c] - Ps[sk * L.ldp + a] * Ps[sj * L.ldp + c];
            else
              pf2 = Qs[(a - n) * L.ldq + sj] * Qs[(c - n) * L.ldq + sk] -
                    Qs[(a - n) * L.ldq + sk] * Qs[(c - n) * L.ldq + sj];
          } else {
            const int u = sa == 0 ? a : c, d = (sa == 0 ? c : a) - n;
            const int ru = sa == 0 ? sj : sk, qd = sa == 0 ? sk : sj;
            pf2 = Ps[ru * L.ldp + u] * Qs[d * L.ldq + qd] -
                  Ws[d * L.ldw + u] * (Ts[ru * L.ldt + qd] - f(ru, qd));
          }
          // second move c: cs -> k after the first, relative to x'
          const double lc2 = G[sk] * occ1(sk, oc) - G[cs] * occ1(cs, oc) +
                             (hs[sk] + V[(int64_t)sk * ns + sj] - V[(int64_t)sk * ns + si]) -
                             (hs[cs] + V[(int64_t)cs * ns + sj] - V[(int64_t)cs * ns + si]) -
                             V[(int64_t)cs * ns + sk];
          r2 = pf2 * exp(lc1 + lc2);
        }
        s2 += -nt[nb2] * r2;
      }
    }
    f2_part += t1amp * s2;
  }
  block_sum2(e_part, f2_part, red);
  if (tid == 0) {
    const double e1 = eu + e_part;
    const int64_t row = I.eloc_off + (int64_t)slot * I.W + lw;
    f1_out[row] = e1;
    f2_out[row] = eu * e1 + f2_part;
  }
}

// Moments of every instance over its first n_used slots, one workgroup per
// instance, fixed-order sums; then alpha_1 from dE_1/dalpha = 0:
//   E_1 = N/D, N = h1 + a (h20 + h11) + a^2 h12, D = 1 + 2 a h1 + a^2 h11,
//   (n2 d1 - n1 d2) a^2 + 2 (n2 d0 - n0 d2) a + (n1 d0 - n0 d1) = 0,
// the root with the lower E_1.  out[k*7 + ...] = h1, h11, h20, h12, alpha, E_1, roots.
__device__ inline double e1_of(const double* h, double a) {
  return (h[0] + a * (h[2] + h[1]) + a * a * h[3]) / (1.0 + 2.0 * a * h[0] + a * a * h[1]);
}

__global__ __launch_bounds__(256) void k_lanczos_moments(Pools P, int n_used,
                                                         const double* __restrict__ f1,
                                                         const double* __restrict__ f2,
                                                         double* __restrict__ out) {
  __shared__ double red[16];
  const InstDev& I = P.inst[blockIdx.x];
  const int64_t rows = (int64_t)n_used * I.W;
  const double* a1 = f1 + I.eloc_off;
  const double* a2 = f2 + I.eloc_off;
  double s1 = 0.0, s11 = 0.0, s20 = 0.0, s12 = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const double x = a1[r], y = a2[r];
    s1 += x;
    s11 += x * x;
    s20 += y;
    s12 += x * y;
  }
  block_sum2(s1, s11, red);
  block_sum2(s20, s12, red);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / (double)rows;
    double h[4] = {s1 * inv, s11 * inv, s20 * inv, s12 * inv};
    const double n0 = h[0], n1 = h[2] + h[1], n2 = h[3], d0 = 1.0, d1 = 2.0 * h[0], d2 = h[1];
    const double qa = n2 * d1 - n1 * d2, qb = 2.0 * (n2 * d0 - n0 * d2), qc = n1 * d0 - n0 * d1;
    double alpha = 0.0;
    int nroot = 0;
    if (qa == 0.0) {
      if (qb != 0.0) {
        alpha = -qc / qb;
        nroot = 1;
      }
    } else {
      const double disc = qb * qb - 4.0 * qa * qc;
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double ra = (-qb + sq) / (2.0 * qa), rb = (-qb - sq) / (2.0 * qa);
        alpha = e1_of(h, rb) < e1_of(h, ra) ? rb : ra;
        nroot = 2;
      }
    }
    double* o = out + (int64_t)blockIdx.x * 7;
    for (int k = 0; k < 4; ++k) o[k] = h[k];
    o[4] = alpha;
    o[5] = e1_of(h, alpha);
    o[6] = (double)nroot;
  }
}
}  // namespace

size_t local_h2_lds_bytes(int ne, int ns) { return h2_layout(ne, ns).total; }

template <typename T>
void launch_local_h2(const Pools& P, const int32_t* wlist, int n, int slot, double* f1,
                     double* f2, int max_ne, int max_ns, hipStream_t s) {
  if (n <= 0) return;
  const size_t sh = h2_layout(max_ne, max_ns).total;
  if (sh > 65536)
    (void)hipFuncSetAttribute((const void*)&k_local_h2<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  hipLaunchKernelGGL((k_local_h2<T>), dim3(n), dim3(kH2Threads), sh, s, P, wlist, slot, f1, f2);
}

void launch_lanczos_moments(const Pools& P, int n_inst, int n_used, const double* f1,
                            const double* f2, double* out, hipStream_t s) {
  if (n_inst <= 0) return;
  hipLaunchKernelGGL(k_lanczos_moments, dim3(n_inst), dim3(256), 0, s, P, n_used, f1, f2, out);
}

template void launch_local_h2<double>(const Pools&, const int32_t*, int, int, double*, double*,
                                      int, int, hipStream_t);
template void launch_local_h2<float>(const Pools&, const int32_t*, int, int, double*, double*,
                                     int, int, hipStream_t);

}  // namespace mvmc
