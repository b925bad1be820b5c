// HIP kernels for one time step of the decoupled scheme (Algorithm 1 / 2) on gfx950.
//
// Data layout (HBM): every nodal field is FP64, value[(p*Ny + iy)*Nx + ix];
// element-local work buffers are value[(p*ne + e)*nq + b*(K+1) + a] with
// e = ey*nx + ex.
//
// Kernel families
//  * element kernels (one work-group per (element, plane)): gather nodal
//    values into LDS, tensor-product (sum-factorised) derivatives with the GLL
//    differentiation matrix, pointwise terms at the GLL quadrature points,
//    and the transposed ("weak divergence") contraction, written to an
//    element-local buffer;
//  * nodal kernels (one thread per node): direct-stiffness summation of the
//    element-local buffers in a fixed order (deterministic, no atomics), plus
//    nodal source and boundary terms;
//  * solve kernels: FP64 residual with the assembled 1D operators, and the two
//    fast-diagonalisation passes  T = (Sy^T R Sx) ./ (ly_i + lx_j + c_p)  and
//    X += Sy T Sx^T, each a chain of two LDS-staged GEMMs per (plane, column
//    block), templated on the compute type (double / float).
#include <climits>
#include <cmath>
#include <functional>
#include <type_traits>
#include <vector>

#include "pfd_internal.h"
#include "pfd_launch.h"

namespace pfd {

#define WG 256

__device__ __forceinline__ int gidx(const Geo& g, int ex, int ey, int a, int b) {
  int ix = ex * g.K + a;
  if (g.periodic && ix == g.Nx) ix = 0;
  return (ey * g.K + b) * g.Nx + ix;
}

// ------------------------------------------------------------------ mixture laws
__device__ __forceinline__ double eps_of(const Par& P, double p) {
  return 0.5 * (P.eps1 + P.eps2) + 0.25 * (P.eps1 - P.eps2) * p * (3.0 - p * p);
}
__device__ __forceinline__ double deps_of(const Par& P, double p) {
  return 0.75 * (P.eps2 - P.eps1) * (p * p - 1.0);
}
__device__ __forceinline__ double h_of(const Par& P, double p) {
  return p * (p * p - 1.0) / (P.eta * P.eta);
}
// Theta'(phi)/lambda with lambda = 3 sigma eta / (2 sqrt 2)
__device__ __forceinline__ double thp_of(const Par& P, double p) {
  return P.cos_theta * (p * p - 1.0) * (0.70710678118654752440 / P.eta);
}

// ---------------------------------------------------------------- element helpers
// shared element context: D and w in LDS, geometry of this element
struct ElemLDS {
  double D[(PFD_KMAX + 1) * (PFD_KMAX + 1)];
  double w[PFD_KMAX + 1];
};

__device__ __forceinline__ void load_gll(const Geo& g, ElemLDS& s) {
  for (int i = threadIdx.x; i < g.nq; i += blockDim.x) s.D[i] = g.D[i];
  for (int i = threadIdx.x; i < g.n; i += blockDim.x) s.w[i] = g.w[i];
}

// x- and y-derivatives of F element arrays f[b*n + p] at local (a,b), in one pass over row b
// and column a: the D entries are read once for all arrays, each sum runs over p = 0..n-1
template <int F>
__device__ __forceinline__ void grad2(const ElemLDS& s, int n, int a, int b, const double* const (&f)[F], double sx,
                                      double sy, double (&dx)[F], double (&dy)[F]) {
#pragma unroll
  for (int i = 0; i < F; ++i) dx[i] = dy[i] = 0.0;
  for (int p = 0; p < n; ++p) {
    const double da = s.D[a * n + p], db = s.D[b * n + p];
#pragma unroll
    for (int i = 0; i < F; ++i) {
      dx[i] += da * f[i][b * n + p];
      dy[i] += db * f[i][p * n + a];
    }
  }
#pragma unroll
  for (int i = 0; i < F; ++i) {
    dx[i] *= sx;
    dy[i] *= sy;
  }
}
// x- and y-parts of the weak divergence in one pass: sum_p D[p][a] gx[b*n+p] and
// sum_p D[p][b] gy[p*n+a] (gx, gy pre-multiplied by the weights)
__device__ __forceinline__ void wdxy(const ElemLDS& s, int n, int a, int b, const double* gx, const double* gy,
                                     double& ox, double& oy) {
  double ax = 0.0, ay = 0.0;
  for (int p = 0; p < n; ++p) {
    ax += s.D[p * n + a] * gx[b * n + p];
    ay += s.D[p * n + b] * gy[p * n + a];
  }
  ox = ax;
  oy = ay;
}

// A work-group takes one element on g.ppw consecutive planes (ppw nq <= 256 threads, so the
// lanes are not left idle at small orders); thread = (sub-plane, local node t).  Element arrays
// in LDS are declared with ELEM_ARRAY and point at the sub-plane's nq-slice.
#define ELEM_LDS_N ((PFD_KMAX + 1) * (PFD_KMAX + 1) > 256 ? (PFD_KMAX + 1) * (PFD_KMAX + 1) : 256)

// The dispatcher hands work-groups to the eight XCDs in turn (linear id mod 8), and each XCD has
// its own L2.  xcd_tile maps a 2D grid's linear id to a logical tile (bx, by), bx fastest, so that
// each XCD takes one contiguous range of logical tiles: neighbouring tiles, which share halo rows
// or element edges, are then read through one L2.  A bijection of the grid for any size.
__device__ __forceinline__ void xcd_tile(const VGrid& vg, int& bx, int& by) {
  constexpr int NXCD = 8;
  const int gx = vg.g.x, total = gx * vg.g.y, lin = vg.b.x + gx * vg.b.y;
  const int q = total / NXCD, r = total - q * NXCD, x = lin % NXCD, j = lin / NXCD;
  const int lb = x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
  by = lb / gx;
  bx = lb - by * gx;
}
// the same with by fastest in the logical order: the tiles of one bx (which share a streamed
// operand block) land on one XCD
__device__ __forceinline__ void xcd_tile_yfast(const VGrid& vg, int& bx, int& by) {
  constexpr int NXCD = 8;
  const int gy = vg.g.y, total = vg.g.x * gy, lin = vg.b.x + vg.g.x * vg.b.y;
  const int q = total / NXCD, r = total - q * NXCD, x = lin % NXCD, j = lin / NXCD;
  const int lb = x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
  bx = lb / gy;
  by = lb - bx * gy;
}

#define ELEM_PROLOGUE                                                    \
  int e, pgrp;                                                           \
  xcd_tile(vg, e, pgrp);                                                     \
  const int ex = e % g.nx, ey = e / g.nx;                                \
  const int n = g.n, nq = g.nq;                                          \
  const int sub = (int)threadIdx.x / nq, t = (int)threadIdx.x - sub * nq; \
  const int pl = pgrp * g.ppw + sub;                                     \
  const bool act = sub < g.ppw && pl < g.planes;                         \
  const int so = act ? sub * nq : 0;                                     \
  const int a = act ? t % n : 0, b = act ? t / n : 0;                    \
  const double hx = g.hx[ex], hy = g.hy[ey];                             \
  const double sx = 2.0 / hx, sy = 2.0 / hy;                             \
  const long pofs = (long)(act ? pl : 0) * g.Ng;                         \
  const int gi = gidx(g, ex, ey, a, b);                                  \
  const long lofs = ((long)(act ? pl : 0) * g.nx * g.ny + e) * nq + t;   \
  __shared__ ElemLDS s;                                                  \
  load_gll(g, s);
#define ELEM_ARRAY(name)                 \
  __shared__ double name##_all[ELEM_LDS_N]; \
  double* const name = name##_all + so;

// ------------------------------------------------------------------ DSS (gather-sum)
// sum of the element-local contributions at global node (ix, iy) of plane pl
__device__ __forceinline__ double dss(const Geo& g, const double* L, int pl, int ix, int iy) {
  // the (at most) two elements along x and along y that hold the node, as (element, local index)
  // pairs with a 0/1 weight; an absent second pair repeats the first with weight 0, so the four
  // loads always issue together (no branch around them) and absent terms add exact zeros
  const int K = g.K;
  int ex0, a0, ex1, a1;
  double wx1;
  if (ix % K == 0) {
    const int ex = ix / K;
    const bool left = g.periodic || ex > 0, right = g.periodic || ex < g.nx;
    const int el = ex == 0 ? g.nx - 1 : ex - 1;   // the left element (wrapped when periodic)
    ex0 = left ? el : ex;
    a0 = left ? K : 0;
    ex1 = ex < g.nx ? ex : el;                    // a node past the last element has only one
    a1 = ex < g.nx ? 0 : K;
    wx1 = (left && right) ? 1.0 : 0.0;
  } else {
    ex0 = ex1 = ix / K;
    a0 = a1 = ix % K;
    wx1 = 0.0;
  }
  int ey0, b0, ey1, b1;
  double wy1;
  if (iy % K == 0) {
    const int ey = iy / K;
    const bool below = ey > 0, above = ey < g.ny;
    ey0 = below ? ey - 1 : ey;
    b0 = below ? K : 0;
    ey1 = above ? ey : ey - 1;
    b1 = above ? 0 : K;
    wy1 = (below && above) ? 1.0 : 0.0;
  } else {
    ey0 = ey1 = iy / K;
    b0 = b1 = iy % K;
    wy1 = 0.0;
  }
  const long base = (long)pl * g.nx * g.ny;
  const double* L00 = L + (base + (long)ey0 * g.nx + ex0) * g.nq + b0 * g.n + a0;
  const double* L01 = L + (base + (long)ey0 * g.nx + ex1) * g.nq + b0 * g.n + a1;
  const double* L10 = L + (base + (long)ey1 * g.nx + ex0) * g.nq + b1 * g.n + a0;
  const double* L11 = L + (base + (long)ey1 * g.nx + ex1) * g.nq + b1 * g.n + a1;
  const double v00 = *L00, v01 = *L01, v10 = *L10, v11 = *L11;
  // same order of the present terms as a loop over (y pair, x pair)
  double acc = 0.0;
  acc += v00;
  acc += wx1 * v01;
  acc += wy1 * v10;
  acc += wy1 * wx1 * v11;
  return acc;
}

#define NODAL_PROLOGUE                                                   \
  const long id = (long)vg.b.x * blockDim.x + threadIdx.x;           \
  if (id >= (long)g.planes * g.Ng) return;                               \
  const int pl = (int)(id / g.Ng);                                       \
  const int node = (int)(id - (long)pl * g.Ng);                          \
  const int iy = node / g.Nx, ix = node - iy * g.Nx;                     \
  (void)pl;

// Right side of a solve and its initial guess.
//  * warm start (Fn != nullptr, FP32-refined path): x0 = extrapolated history
//    cs_n Fn + cs_o Fo (Dirichlet data on Dirichlet nodes), so the low-precision
//    corrections act on a small residual; the solve computes the first residual, or (L.bprev,
//    right sides of the two previous steps kept) it is formed here from them.
//  * cold start (FP64 path): x0 = Dirichlet data x_D, zero elsewhere, and the first
//    residual r = b - A x_D is folded in here: each family's Dirichlet set is a union of
//    whole sides, so (A x_D) at a free node needs only the first and last columns of the
//    1D stiffness matrices (Kx0 = Kx[:,0], KxN = Kx[:,Nx-1], likewise in y).
// Dirichlet node of a family (gap nodes of a partial electrode row are unknowns)
__device__ __forceinline__ bool is_dir(const unsigned char* dirx, const unsigned char* diry,
                                       const unsigned char* ebot, int ix, int iy) {
  // the flag loads are issued together (ebot is the same for every thread: null or not)
  const bool dxi = dirx[ix] != 0, dyi = diry[iy] != 0;
  const bool gap = ebot && ebot[ix] == 0 && iy == 0;   // bottom-row gap node of an electrode set
  return dxi || (dyi && !gap);
}

__device__ __forceinline__ void rhs_out(const Geo& g, const Par& P, const Lift& L, const double* gD,
                                        const double* Fn, const double* Fo, long id, long pofs, int ix, int iy,
                                        double b, double* bb, double* r, double* x0) {
  const double bo = L.bprev ? bb[id] : 0.0;   // b^{n-1}, in the slot that now takes b^{n+1}
  bb[id] = b;
  const bool dn = is_dir(L.dirx, L.diry, L.ebot, ix, iy);
  const double gd = gD ? gD[id] : 0.0;   // (no Dirichlet data: no Dirichlet node)
  if (Fn) {
    const double fn = Fn[id], fo = Fo[id];
    x0[id] = dn ? gd : P.cs_n * fn + P.cs_o * fo;
    // recycled first residual: A x^n = b^n, A x^{n-1} = b^{n-1} and the Dirichlet data did not
    // change, so b - A x0 = b - (cs_n b^n + cs_o b^{n-1}) on free nodes
    if (L.bprev) r[id] = dn ? 0.0 : b - (P.cs_n * L.bprev[id] + P.cs_o * bo);
    return;
  }
  if (dn) {
    r[id] = 0.0;
    x0[id] = gd;
    return;
  }
  double ax = 0.0, ay = 0.0;
  if (gD) {
    // lift of the Dirichlet sides: every term loaded (the coupling columns and the data exist
    // for every side), the flags only select, so no load waits behind a flag
    const bool dx0 = L.dirx[0] != 0, dxN = L.dirx[g.Nx - 1] != 0, dyN = L.diry[g.Ny - 1] != 0;
    const bool dy0 = L.diry[0] != 0 && iy > 0 && (!L.ebot || L.ebot[ix]);
    const double t0 = L.Kx0[ix] * gD[pofs + (long)iy * g.Nx];
    const double tN = L.KxN[ix] * gD[pofs + (long)iy * g.Nx + g.Nx - 1];
    const double s0 = L.Ky0[iy] * gD[pofs + ix];
    const double sN = L.KyN[iy] * gD[pofs + (long)(g.Ny - 1) * g.Nx + ix];
    if (dx0) ax += t0;
    if (dxN) ax += tN;
    if (dy0) ay += s0;
    if (dyN) ay += sN;
  }
  if (L.ebot && iy == 0) {  // gap node: coupling along the bottom row to the electrode nodes
    for (int d = -g.K; d <= g.K; ++d) {
      int j = ix + d;
      if (g.periodic) j = (j < 0) ? j + g.Nx : (j >= g.Nx ? j - g.Nx : j);
      else if (j < 0 || j >= g.Nx) continue;
      if (L.ebot[j] && !L.dirx[j]) ax += L.KxB[(long)(d + g.K) * g.Nx + ix] * gD[pofs + j];
    }
  }
  r[id] = b - (ax * L.My[iy] + L.Mx[ix] * ay);
  x0[id] = 0.0;
}

// =================================================================== stage V (eq. 54)
// L0 = -int (eps(phi*) - eps0) grad V* . grad e   (element-local)
__device__ __forceinline__ void k_V_elem_run(const VGrid& vg, Geo g, Par P, const double* phn, const double* pho,
                                             const double* Vn, const double* Vo, double* L0) {
  ELEM_PROLOGUE
  ELEM_ARRAY(sV)
  ELEM_ARRAY(sgx)
  ELEM_ARRAY(sgy)
  double phs = 0.0;
  if (act) {
    sV[t] = P.cs_n * Vn[pofs + gi] + P.cs_o * Vo[pofs + gi];
    phs = P.cs_n * phn[pofs + gi] + P.cs_o * pho[pofs + gi];
  }
  __syncthreads();
  if (act) {
    double r = eps_of(P, phs) - P.eps0;
    const double* f[1] = {sV};
    double dx[1], dy[1];
    grad2<1>(s, n, a, b, f, sx, sy, dx, dy);
    sgx[t] = s.w[a] * r * dx[0];
    sgy[t] = s.w[b] * r * dy[0];
  }
  __syncthreads();
  if (act) {
    double wx, wy;
    wdxy(s, n, a, b, sgx, sgy, wx, wy);
    L0[lofs] = -(0.5 * hy * s.w[b] * wx + 0.5 * hx * s.w[a] * wy);
  }
}
struct k_V_elem : KDef<&k_V_elem_run, WG, 0> {};

// b = (DSS(L0) - M f_V)/eps0, Dirichlet values from VD
__device__ __forceinline__ void k_V_rhs_run(const VGrid& vg, Geo g, Par P, Lift L, const double* L0,
                                            const double* Mdiag, const double* fV, const double* Vd, const double* Fn,
                                            const double* Fo, double* bb, double* r, double* x0) {
  NODAL_PROLOGUE
  const double v = dss(g, L0, pl, ix, iy) - Mdiag[node] * fV[id];
  rhs_out(g, P, L, Vd, Fn, Fo, id, (long)pl * g.Ng, ix, iy, v / P.eps0, bb, r, x0);
}
struct k_V_rhs : KDef<&k_V_rhs_run, 0, 0> {};

// =================================================================== stage E (eq. 55)
__device__ __forceinline__ void k_E_elem_run(const VGrid& vg, Geo g, const double* V, double* L0, double* L1) {
  ELEM_PROLOGUE
  ELEM_ARRAY(sV)
  if (act) sV[t] = V[pofs + gi];
  __syncthreads();
  if (act) {
    double wq = 0.25 * hx * hy * s.w[a] * s.w[b];
    const double* f[1] = {sV};
    double dx[1], dy[1];
    grad2<1>(s, n, a, b, f, sx, sy, dx, dy);
    L0[lofs] = wq * dx[0];
    L1[lofs] = wq * dy[0];
  }
}
struct k_E_elem : KDef<&k_E_elem_run, WG, 0> {};

__device__ __forceinline__ void k_E_nodal_run(const VGrid& vg, Geo g, const double* L0, const double* L1,
                                              const double* Mdiag, const double* Ez, double* Ex, double* Ey,
                                              double* E2) {
  NODAL_PROLOGUE
  double m = Mdiag[node];
  double ex = dss(g, L0, pl, ix, iy) / m, ey = dss(g, L1, pl, ix, iy) / m;
  Ex[id] = ex;
  Ey[id] = ey;
  double ez = Ez ? Ez[id] : 0.0;
  E2[id] = ex * ex + ey * ey + ez * ez;
}
struct k_E_nodal : KDef<&k_E_nodal_run, 0, 0> {};

// =================================================================== stage psi (eq. 56)
// L0 = -int Q1 w + int grad Q2 . grad w ;  Q2 also written (nodal, same at shared nodes)
__device__ __forceinline__ void k_psi_elem_run(const VGrid& vg, Geo g, Par P, const double* phn, const double* pho,
                                               const double* uxn, const double* uxo, const double* uyn,
                                               const double* uyo, const double* E2, const double* gsrc,
                                               const double* uzn, const double* uzo, const double* dzphs,
                                               double* L0) {
  ELEM_PROLOGUE
  ELEM_ARRAY(sph)
  ELEM_ARRAY(sQ2)
  ELEM_ARRAY(sgx)
  ELEM_ARRAY(sgy)
  double phh = 0.0, uxs = 0.0, uys = 0.0, gg = 0.0;
  if (act) {
    double pn = phn[pofs + gi], po = pho[pofs + gi];
    double phs = P.cs_n * pn + P.cs_o * po;
    phh = P.ch_n * pn + P.ch_o * po;
    sph[t] = phs;
    sQ2[t] = h_of(P, phs) - P.S / (P.eta * P.eta) * phs - deps_of(P, phs) * E2[pofs + gi] / (2.0 * P.lam);
    uxs = P.cs_n * uxn[pofs + gi] + P.cs_o * uxo[pofs + gi];
    uys = P.cs_n * uyn[pofs + gi] + P.cs_o * uyo[pofs + gi];
    gg = gsrc[pofs + gi];
  }
  // 3D: u*_z d(phi*)/dz (the z-derivative taken from the spectral phi), loaded before the barrier
  double uzd = 0.0;
  if (uzn && act) {
    const long id = pofs + gi;
    uzd = (P.cs_n * uzn[id] + P.cs_o * uzo[id]) * dzphs[id];
  }
  __syncthreads();
  double q1 = 0.0;
  if (act) {
    const double* f[2] = {sph, sQ2};
    double dx[2], dy[2];
    grad2<2>(s, n, a, b, f, sx, sy, dx, dy);
    double adv = uxs * dx[0] + uys * dy[0];
    if (uzn) adv += uzd;
    q1 = (gg - adv + phh / P.dt) / (P.lam * P.gamma1);
    sgx[t] = s.w[a] * dx[1];
    sgy[t] = s.w[b] * dy[1];
  }
  __syncthreads();
  if (act) {
    double wq = 0.25 * hx * hy * s.w[a] * s.w[b];
    double wx, wy;
    wdxy(s, n, a, b, sgx, sgy, wx, wy);
    L0[lofs] = -wq * q1 + 0.5 * hy * s.w[b] * wx + 0.5 * hx * s.w[a] * wy;
  }
}
struct k_psi_elem : KDef<&k_psi_elem_run, WG, 0> {};

// b_psi = DSS(L0) + Bo (g1 + c_psi g2) + Bs (g1 + c_psi U);  U = -g3 - Theta'(phi*)/lambda
// also stores U (reused by the phi stage) and x0 = psi*
__device__ __forceinline__ void k_psi_rhs_run(const VGrid& vg, Geo g, Par P, const double* L0, const double* bmo,
                                              const double* bmw, const double* g1, const double* g2, const double* g3,
                                              const double* phn, const double* pho, const double* E2,
                                              const double* Fn, const double* Fo, double* bb, double* U, double* Q2,
                                              double* r, double* x0, const double* bprev) {
  NODAL_PROLOGUE
  double phs = P.cs_n * phn[id] + P.cs_o * pho[id];
  double u = -g3[id] - thp_of(P, phs);
  U[id] = u;
  Q2[id] = h_of(P, phs) - P.S / (P.eta * P.eta) * phs - deps_of(P, phs) * E2[id] / (2.0 * P.lam);
  const double v = dss(g, L0, pl, ix, iy) + bmo[node] * (g1[id] + P.c_psi * g2[id]) +
                   bmw[node] * (g1[id] + P.c_psi * u);
  const double bo = bprev ? bb[id] : 0.0;   // recycled first residual (as rhs_out)
  bb[id] = v;  // no Dirichlet node: cold start r = b, x0 = 0
  if (Fn) {
    x0[id] = P.cs_n * Fn[id] + P.cs_o * Fo[id];
    if (bprev) r[id] = v - (P.cs_n * bprev[id] + P.cs_o * bo);
  } else {
    r[id] = v;
    x0[id] = 0.0;
  }
}
struct k_psi_rhs : KDef<&k_psi_rhs_run, 0, 0> {};

// =================================================================== stage phi (eq. 57)
__device__ __forceinline__ void k_phi_rhs_run(const VGrid& vg, Geo g, Par P, const double* Mdiag, const double* psi,
                                              const double* bmo, const double* bmw, const double* g2, const double* U,
                                              const double* Fn, const double* Fo, double* bb, double* r, double* x0,
                                              const double* bprev) {
  NODAL_PROLOGUE
  const double v = -Mdiag[node] * psi[id] + bmo[node] * g2[id] + bmw[node] * U[id];
  const double bo = bprev ? bb[id] : 0.0;   // recycled first residual (as rhs_out)
  bb[id] = v;  // no Dirichlet node
  if (Fn) {
    x0[id] = P.cs_n * Fn[id] + P.cs_o * Fo[id];
    if (bprev) r[id] = v - (P.cs_n * bprev[id] + P.cs_o * bo);
  } else {
    r[id] = v;
    x0[id] = 0.0;
  }
}
struct k_phi_rhs : KDef<&k_phi_rhs_run, 0, 0> {};

// optional 3D inputs / outputs of the momentum element kernel (Algorithm 2):
// z-derivatives come from the spectral representation (nodal values, one per node)
struct Mom3 {
  const double *uzn, *uzo, *dzphi, *dzPhi, *dzux, *dzuy, *dzuz, *dzP, *fz;
  double *LBP, *LAz, *LBx, *LBy;
};

// =================================================================== momentum terms (eq. 49)
// L0 = rho0 int G.grad q - rho0 int_dOmega (mu/rho) (n x w*).grad q   (pressure, eqs. 58a / 77a)
// L1, L2 = (1/nu_m)[int G v -+ int K x grad v] - (1/nu_m) int_open L v (velocity, eqs. 59a / 78a;
//          the -grad P^{n+1}/rho0 part is added after the pressure solve)
// 3D (Z3): the parts multiplied by i beta_k in the per-mode forms go to LBP, LBx, LBy, and the
//          z velocity right side to LAz (G, omega*, K are full 3-vectors there).
template <bool Z3>
__device__ __forceinline__ void k_mom_elem_run(const VGrid& vg, Geo g, Par P, const double* phi, const double* psi,
                                               const double* E2, const double* Q2, const double* uxn,
                                               const double* uxo, const double* uyn, const double* uyo,
                                               const double* Pn, const double* Po, const double* fx, const double* fy,
                                               double* L0, double* L1, double* L2, Mom3 z) {
  ELEM_PROLOGUE
  ELEM_ARRAY(sph)
  ELEM_ARRAY(sPhi)
  ELEM_ARRAY(sux)
  ELEM_ARRAY(suy)
  ELEM_ARRAY(suz)
  ELEM_ARRAY(sP)
  ELEM_ARRAY(sgx)
  ELEM_ARRAY(sgy)
  ELEM_ARRAY(sKz)
  ELEM_ARRAY(sfz)
  ELEM_ARRAY(sfx)
  ELEM_ARRAY(sfy)
  double ph = 0.0, ps = 0.0, e2 = 0.0, uh[3] = {0.0, 0.0, 0.0}, ff[3] = {0.0, 0.0, 0.0};
  if (act) {
    const long id = pofs + gi;
    ph = phi[id];
    ps = psi[id];
    e2 = E2[id];
    sph[t] = ph;
    sPhi[t] = ps - P.c_psi * ph - Q2[id];
    double un = uxn[id], uo = uxo[id];
    sux[t] = P.cs_n * un + P.cs_o * uo;
    uh[0] = P.ch_n * un + P.ch_o * uo;
    un = uyn[id];
    uo = uyo[id];
    suy[t] = P.cs_n * un + P.cs_o * uo;
    uh[1] = P.ch_n * un + P.ch_o * uo;
    if (Z3) {
      un = z.uzn[id];
      uo = z.uzo[id];
      suz[t] = P.cs_n * un + P.cs_o * uo;
      uh[2] = P.ch_n * un + P.ch_o * uo;
      ff[2] = z.fz[id];
    } else {
      suz[t] = 0.0;
    }
    sP[t] = P.cs_n * Pn[id] + P.cs_o * Po[id];
    ff[0] = fx[id];
    ff[1] = fy[id];
  }
  // the z-derivatives (3D) are requested before the barrier: in flight during the x, y sums
  double zphi = 0.0, zPhi = 0.0, zux = 0.0, zuy = 0.0, zuz = 0.0, zP = 0.0;
  if (Z3 && act) {
    const long id = pofs + gi;
    zphi = z.dzphi[id];
    zPhi = z.dzPhi[id];
    zux = z.dzux[id];
    zuy = z.dzuy[id];
    zuz = z.dzuz[id];
    zP = z.dzP[id];
  }
  __syncthreads();
  double G[3] = {0.0, 0.0, 0.0}, Kv[3] = {0.0, 0.0, 0.0}, om[3] = {0.0, 0.0, 0.0}, mr = 0.0;
  if (act) {
    const long id = pofs + gi;
    const double pc = fmin(1.0, fmax(-1.0, ph));
    const double rho = 0.5 * (P.rho1 + P.rho2) + 0.5 * (P.rho1 - P.rho2) * pc;
    const double mu = 0.5 * (P.mu1 + P.mu2) + 0.5 * (P.mu1 - P.mu2) * pc;
    const double irho = 1.0 / rho;
    const double drr = 0.5 * (P.rho1 - P.rho2), dmm = 0.5 * (P.mu1 - P.mu2);
    // x, y derivatives of phi*, Phi, u*_x, u*_y, P*, u*_z
    constexpr int NF = Z3 ? 6 : 5;
    const double* fl[NF];
    fl[0] = sph; fl[1] = sPhi; fl[2] = sux; fl[3] = suy; fl[4] = sP;
    if (Z3) fl[NF - 1] = suz;
    double dX[NF], dY[NF];
    grad2<NF>(s, n, a, b, fl, sx, sy, dX, dY);
    const double gph[3] = {dX[0], dY[0], zphi};
    const double cnu = (rho * dmm - mu * drr) * irho * irho;  // grad(mu/rho) = cnu grad(phi)
    const double jc = 0.5 * (P.rho1 - P.rho2) * P.lam * P.gamma1;
    const double Jt[3] = {jc * dX[1], jc * dY[1], Z3 ? jc * zPhi : 0.0};
    const double u[3] = {sux[t], suy[t], suz[t]};
    // gu[i][k] = d_i u*_k
    double gu[3][3];
    gu[0][0] = dX[2];
    gu[0][1] = dX[3];
    gu[1][0] = dY[2];
    gu[1][1] = dY[3];
    if (Z3) {
      gu[0][2] = dX[NF - 1];
      gu[1][2] = dY[NF - 1];
      gu[2][0] = zux;
      gu[2][1] = zuy;
      gu[2][2] = zuz;
    } else {
      gu[0][2] = gu[1][2] = gu[2][0] = gu[2][1] = gu[2][2] = 0.0;
    }
    om[0] = gu[1][2] - gu[2][1];
    om[1] = gu[2][0] - gu[0][2];
    om[2] = gu[0][1] - gu[1][0];
    const double lap = ps - P.alpha * ph;
    const double dep = deps_of(P, ph);
    const double gP[3] = {dX[4], dY[4], zP};
    const double cP = 1.0 / P.rho0 - irho;
    const double gnu[3] = {cnu * gph[0], cnu * gph[1], cnu * gph[2]};
    const double cr[3] = {gnu[1] * om[2] - gnu[2] * om[1], gnu[2] * om[0] - gnu[0] * om[2],
                          gnu[0] * om[1] - gnu[1] * om[0]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (!Z3 && k == 2) break;
      double gmD = 0.0, Nk = 0.0, JU = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        gmD += dmm * gph[i] * (gu[i][k] + gu[k][i]);
        Nk += u[i] * gu[i][k];
        JU += Jt[i] * gu[i][k];
      }
      const double T = (ff[k] - P.lam * lap * gph[k] - 0.5 * dep * e2 * gph[k] + gmD - JU) * irho +
                       uh[k] / P.dt - Nk + cP * gP[k];
      G[k] = T + cr[k];
    }
    mr = mu * irho;
#pragma unroll
    for (int k = 0; k < 3; ++k) Kv[k] = (mr - P.nu_m) * om[k];
    sgx[t] = s.w[a] * G[0];
    sgy[t] = s.w[b] * G[1];
    sKz[t] = Kv[2];
    sfz[t] = mr * om[2];
    sfx[t] = Kv[0];
    sfy[t] = Kv[1];
  }
  __syncthreads();
  if (act) {
    const double wq = 0.25 * hx * hy * s.w[a] * s.w[b];
    const double ewx = 0.5 * hx * s.w[a], ewy = 0.5 * hy * s.w[b];   // edge weights
    // weak divergence of G (x, y parts) and of the K components (K weighted by w_p inside),
    // one pass over row b and column a
    double gdx = 0.0, gdy = 0.0, kz_y = 0.0, kz_x = 0.0, ky_x = 0.0, kx_y = 0.0;
    for (int p = 0; p < n; ++p) {
      const double dpa = s.D[p * n + a], dpb = s.D[p * n + b], wp = s.w[p];
      gdx += dpa * sgx[b * n + p];
      gdy += dpb * sgy[p * n + a];
      kz_y += dpb * wp * sKz[p * n + a];
      kz_x += dpa * wp * sKz[b * n + p];
      if (Z3) {
        ky_x += dpa * wp * sfy[b * n + p];
        kx_y += dpb * wp * sfx[p * n + a];
      }
    }
    double l0 = P.rho0 * (ewy * gdx + ewx * gdy);
    double l1 = wq * G[0] + ewx * kz_y;
    double l2 = wq * G[1] - ewy * kz_x;
    double laz = 0.0, lbp = 0.0;
    if (Z3) {
      laz = wq * G[2] + ewy * ky_x - ewx * kx_y;
      lbp = -P.rho0 * wq * G[2];
    }
    // boundary edges: tangential term of the pressure equation on every side (reading R-Pbnd),
    // its z part (3D), and the L term of the velocity equation on open sides
    const int K = g.K;
    if (ey == 0 && b == 0) {  // bottom, n = (0,-1)
      double acc = 0.0;
      for (int p = 0; p < n; ++p) acc += s.w[p] * sfz[p] * s.D[p * n + a];
      l0 += P.rho0 * acc;
      if (Z3) lbp += P.rho0 * ewx * mr * om[0];
      if (g.side_type[PFD_BOTTOM] == PFD_OPEN) {
        l1 += ewx * Kv[2];
        if (Z3) laz -= ewx * Kv[0];
      }
    }
    if (ey == g.ny - 1 && b == K) {  // top, n = (0,1)
      double acc = 0.0;
      for (int p = 0; p < n; ++p) acc += s.w[p] * sfz[K * n + p] * s.D[p * n + a];
      l0 -= P.rho0 * acc;
      if (Z3) lbp -= P.rho0 * ewx * mr * om[0];
      if (g.side_type[PFD_TOP] == PFD_OPEN) {
        l1 -= ewx * Kv[2];
        if (Z3) laz += ewx * Kv[0];
      }
    }
    if (!g.periodic && ex == 0 && a == 0) {  // left, n = (-1,0)
      double acc = 0.0;
      for (int p = 0; p < n; ++p) acc += s.w[p] * sfz[p * n] * s.D[p * n + b];
      l0 -= P.rho0 * acc;
      if (Z3) lbp -= P.rho0 * ewy * mr * om[1];
      if (g.side_type[PFD_LEFT] == PFD_OPEN) {
        l2 -= ewy * Kv[2];
        if (Z3) laz += ewy * Kv[1];
      }
    }
    if (!g.periodic && ex == g.nx - 1 && a == K) {  // right, n = (1,0)
      double acc = 0.0;
      for (int p = 0; p < n; ++p) acc += s.w[p] * sfz[p * n + K] * s.D[p * n + b];
      l0 += P.rho0 * acc;
      if (Z3) lbp += P.rho0 * ewy * mr * om[1];
      if (g.side_type[PFD_RIGHT] == PFD_OPEN) {
        l2 += ewy * Kv[2];
        if (Z3) laz -= ewy * Kv[1];
      }
    }
    L0[lofs] = l0;
    L1[lofs] = l1 / P.nu_m;
    L2[lofs] = l2 / P.nu_m;
    if (Z3) {
      z.LBP[lofs] = lbp;
      z.LAz[lofs] = laz / P.nu_m;
      z.LBx[lofs] = wq * Kv[1] / P.nu_m;
      z.LBy[lofs] = -wq * Kv[0] / P.nu_m;
    }
  }
}
template <bool Z3>
struct k_mom_elem : KDef<&k_mom_elem_run<Z3>, WG, 0> {};

// b_P = DSS(L0) - rho0 gamma0/dt sum_walls int (n.w) q ;  x0 = P* (f2 on open sides)
__device__ __forceinline__ void k_P_rhs_run(const VGrid& vg, Geo g, Par P, Lift L, const double* L0, const double* wx,
                                            const double* wy, const double* f2, const double* Fn, const double* Fo,
                                            double* bb, double* r, double* x0) {
  NODAL_PROLOGUE
  double v = dss(g, L0, pl, ix, iy);
  const double c = P.rho0 * P.gamma0 / P.dt;
  const double nw[4] = {-wy[id], wy[id], -wx[id], wx[id]};  // n.w for bottom, top, left, right
  for (int sd = 0; sd < 4; ++sd)
    if (g.side_type[sd] == PFD_WALL) v -= c * g.bm_side[sd][node] * nw[sd];
  rhs_out(g, P, L, f2, Fn, Fo, id, (long)pl * g.Ng, ix, iy, v, bb, r, x0);
}
struct k_P_rhs : KDef<&k_P_rhs_run, 0, 0> {};

// u right side: add -(1/(nu_m rho0)) int grad P^{n+1} v to L1, L2 (and to LAz in 3D, with the
// z-derivative dzP taken from the spectral pressure)
__device__ __forceinline__ void k_gradP_elem_run(const VGrid& vg, Geo g, Par P, const double* Pnew, const double* dzP,
                                                 double* L1, double* L2, double* LAz) {
  ELEM_PROLOGUE
  ELEM_ARRAY(sP)
  // the element-local sums this kernel adds to (and the 3D z-derivative) are requested before
  // the barrier, so they arrive while the x, y derivatives are formed
  double l1 = 0.0, l2 = 0.0, laz = 0.0, dzp = 0.0;
  if (act) {
    sP[t] = Pnew[pofs + gi];
    l1 = L1[lofs];
    l2 = L2[lofs];
    if (dzP) {
      laz = LAz[lofs];
      dzp = dzP[pofs + gi];
    }
  }
  __syncthreads();
  if (act) {
    const double c = -0.25 * hx * hy * s.w[a] * s.w[b] / (P.nu_m * P.rho0);
    const double* f[1] = {sP};
    double dx[1], dy[1];
    grad2<1>(s, n, a, b, f, sx, sy, dx, dy);
    L1[lofs] = l1 + c * dx[0];
    L2[lofs] = l2 + c * dy[0];
    if (dzP) LAz[lofs] = laz + c * dzp;
  }
}
struct k_gradP_elem : KDef<&k_gradP_elem_run, WG, 0> {};

// b_u = DSS(L) + Bo f1 ; x0 = u* with w on walls (two components)
__device__ __forceinline__ void k_u_rhs_run(const VGrid& vg, Geo g, Par P, Lift L, const double* L1, const double* L2,
                                            const double* bmo, const double* f1x, const double* f1y, const double* wx,
                                            const double* wy, const double* Fxn, const double* Fxo, const double* Fyn,
                                            const double* Fyo, double* bx, double* by, double* rx, double* ry,
                                            double* x0x, double* x0y) {
  NODAL_PROLOGUE
  const long pofs = (long)pl * g.Ng;
  Lift Ly = L;   // the y component's history follows the x component's (contiguous blocks)
  if (Ly.bprev) Ly.bprev += (long)g.planes * g.Ng;
  rhs_out(g, P, L, wx, Fxn, Fxo, id, pofs, ix, iy, dss(g, L1, pl, ix, iy) + bmo[node] * f1x[id], bx, rx, x0x);
  rhs_out(g, P, Ly, wy, Fyn, Fyo, id, pofs, ix, iy, dss(g, L2, pl, ix, iy) + bmo[node] * f1y[id], by, ry, x0y);
}
struct k_u_rhs : KDef<&k_u_rhs_run, 0, 0> {};

__device__ __forceinline__ void k_fill_run(const VGrid& vg, long N, double* f, double v) {
  const long i = (long)vg.b.x * blockDim.x + threadIdx.x;
  if (i < N) f[i] = v;
}
struct k_fill : KDef<&k_fill_run, 0, 0> {};

// non-finite guard on a field: sets status[0]
// sticky non-finite flag over f (and f2 when given), one launch
__device__ __forceinline__ void k_check_finite_run(const VGrid& vg, long N, const double* f, const double* f2,
                                                   int* status) {
  long i = (long)vg.b.x * blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < N; i += (long)vg.g.x * blockDim.x) {
    if (!isfinite(f[i])) bad = true;
    if (f2 && !isfinite(f2[i])) bad = true;
  }
  if (bad) atomicOr(status, 1);
}
struct k_check_finite : KDef<&k_check_finite_run, 0, 0> {};

// =================================================================== solves
// Convergence test of the iterative refinement, taken on every FP64 residual r = b - A x the
// refined path forms.  The stop rule is the normwise backward error of x with respect to
// perturbations of A (Rigal & Gaches 1967 with the right side held exact):
//   eta = ||r||_2 / (||A||_2 ||x||_2) <= tol
// over the free nodes of every plane (and stacked component) of the solve, with the per-plane
// bound ||A_p||_2 <= max(Mx) max(My) (max lx + max ly + c_p) from the 1D eigenvalues.  (With
// b = A x up to r, ||b|| <= ||A|| ||x|| + ||r||, so eta is within a factor 2 of the variant
// with ||b|| added to the denominator; two sums keep the fused residual kernel within its
// register budget.)  Each work-group of a residual kernel reduces its nodes' r^2 and
// ||A_p||^2 x^2 (wavefront shuffles, then the four waves in order) and stores the two sums;
// k_chk_decide, launched next, adds them in work-group order (so the result does not depend on
// scheduling), decides, and writes the gate the rest of the solve's kernels read: 1 =
// converged, return at once.  (The kernel boundary publishes the partial sums; a
// per-work-group device-scope release would write back the whole L2 of its XCD every time.)
struct Chk {
  double* part;          // [work-groups][2] partial sums (nullptr: no test)
  const int* gin;        // read on entry: a set gate skips the launch (nullptr: not gated)
  const double* anorm;   // per plane bound of ||A_p||_2 (stacked components repeat it)
  int nplane;            // planes per component (anorm index = plane % nplane)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// two block sums in a fixed order (every thread gets them); red: 2 doubles per wave of LDS
__device__ __forceinline__ void block_sum2(double& a, double& x, double* red) {
  a = wave_sum(a);
  x = wave_sum(x);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = x;
  }
  __syncthreads();
  a = x = 0.0;
  for (int i = 0; i < nw; ++i) {
    a += red[2 * i];
    x += red[2 * i + 1];
  }
  __syncthreads();
}

// Called by every thread of a residual work-group after its nodes were summed into
// (r2, ax2): the work-group's partial sums
__device__ void chk_store(const VGrid& vg, const Chk& ck, double r2, double ax2) {
  __shared__ double red[32];
  block_sum2(r2, ax2, red);
  if (threadIdx.x == 0) {
    const long bid = vg.b.x + (long)vg.g.x * vg.b.y;
    ck.part[2 * bid] = r2;
    ck.part[2 * bid + 1] = ax2;
  }
}

// One work-group: the test of the nblk partial sums the residual kernel before it stored.
// stat (family record): corrections, eta, max corrections, failed solves; status[1] gets bit
// fam when the test after the last allowed correction fails.
__device__ __forceinline__ void k_chk_decide_run(const VGrid& vg, const double* __restrict__ part, long nblk,
                                                 const int* __restrict__ gin, int* __restrict__ gate,
                                                 double* __restrict__ stat, int* __restrict__ status, double tol,
                                                 int it, int last, int fam) {
  if (gin && *gin) return;
  __shared__ double red[32];
  double R = 0.0, X = 0.0;
  for (long i = threadIdx.x; i < nblk; i += blockDim.x) {
    R += part[2 * i];
    X += part[2 * i + 1];
  }
  block_sum2(R, X, red);
  if (threadIdx.x == 0) {
    const double eta = X > 0.0 ? sqrt(R / X) : (R > 0.0 ? HUGE_VAL : 0.0);
    const bool conv = eta <= tol;
    *gate = conv ? 1 : 0;
    stat[1] = eta;
    if (conv || last) {
      stat[0] = it;
      stat[2] = fmax(stat[2], (double)it);
      if (!conv) {
        stat[3] += 1.0;
        atomicOr(status + 1, 1 << fam);
      }
    }
  }
}
struct k_chk_decide : KDef<&k_chk_decide_run, 256, 0> {};

// Copies n values into LDS with U independent loads in flight per thread: value(idx) is read for
// every idx < n (the caller clamps addresses and masks values, so there is no branch around a
// load) and store(idx, v) writes it.  Indices past n are clamped to n - 1, whose value is then
// written twice (the same value), so neither loads nor stores sit under a branch.  A plain
// strided loop would wait for each load in turn.
template <int NT, int U, class T, class Value, class Store>
__device__ __forceinline__ void stage_lds(int n, Value value, Store store) {
  for (int base = 0; base < n; base += NT * U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + (int)threadIdx.x + NT * u;
      v[u] = value(idx < n ? idx : n - 1);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = base + (int)threadIdx.x + NT * u;
      store(idx < n ? idx : n - 1, v[u]);
    }
  }
}

// r = b - (Kx (x) My + Mx (x) Ky + c_p Mx (x) My) x on free nodes, 0 on Dirichlet nodes.
// The 1D stiffness matrices are stored banded and transposed: KxB[(d+K)*Nx + ix] =
// Kx[ix][ix+d] (periodic wrap in x; zero outside the band), so consecutive threads read
// consecutive coefficients.  apply_only = 1 computes y = A x on every node.
template <int K>
__device__ __forceinline__ void k_residual_run(const VGrid& vg, int Nx, int Ny, int planes, int perx,
                                               const double* __restrict__ KxB, const double* __restrict__ Mx,
                                               const unsigned char* __restrict__ dirx, const double* __restrict__ KyB,
                                               const double* __restrict__ My, const unsigned char* __restrict__ diry,
                                               const double* __restrict__ shift, const double* __restrict__ bb,
                                               const double* __restrict__ x, double* __restrict__ r, int apply_only,
                                               const unsigned char* __restrict__ ebot, Chk ck, int kr) {
  if (ck.gin && *ck.gin) return;
  const int KK = K > 0 ? K : kr;   // K = 0: the order is the runtime argument kr
  const long Ng = (long)Nx * Ny;
  const long id0 = (long)vg.b.x * blockDim.x + threadIdx.x;
  double r2 = 0.0, ax2 = 0.0;
  if (id0 < planes * Ng) {
  const long id = id0;
  const int pl = (int)(id / Ng);
  const int node = (int)(id - pl * Ng);
  const int iy = node / Nx, ix = node - iy * Nx;
  const double* xp = x + pl * Ng;
  const double* xrow = xp + (long)iy * Nx;
  // neighbour indices are clamped, not skipped: the band coefficients outside the operator are
  // zero, and with no branch around them all 4K+2 loads are issued together
  double ax = 0.0, ay = 0.0;
#pragma unroll
  for (int d = -KK; d <= KK; ++d) {
    int j = ix + d;
    if (perx) j = (j < 0) ? j + Nx : (j >= Nx ? j - Nx : j);
    else j = (j < 0) ? 0 : (j >= Nx ? Nx - 1 : j);
    ax += KxB[(long)(d + KK) * Nx + ix] * xrow[j];
  }
#pragma unroll
  for (int d = -KK; d <= KK; ++d) {
    int j = iy + d;
    j = (j < 0) ? 0 : (j >= Ny ? Ny - 1 : j);
    ay += KyB[(long)(d + KK) * Ny + iy] * xp[(long)j * Nx + ix];
  }
  const double xv = xrow[ix];
  const double Av = ax * My[iy] + Mx[ix] * ay + shift[pl] * Mx[ix] * My[iy] * xv;
  if (apply_only) {
    r[id] = Av;
  } else {
    const bool dn = is_dir(dirx, diry, ebot, ix, iy);
    const double bv = bb[id];
    const double v = dn ? 0.0 : bv - Av;
    r[id] = v;
    if (ck.part && !dn) {
      const double an = ck.anorm[pl % ck.nplane];
      r2 = v * v;
      ax2 = an * an * xv * xv;
    }
  }
  }
  if (ck.part) chk_store(vg, ck, r2, ax2);
}
template <int K>
struct k_residual : KDef<&k_residual_run<K>, WG, 0> {};

// LDS-tiled variant of k_residual: a work-group takes RROWS rows of one plane; the rows
// iy0-K .. iy0+RROWS-1+K of x are staged in LDS once (coalesced), each with K halo entries on
// either side (the periodic images in x, else zeros, which meet zero band coefficients), so the
// x-neighbours of column ix sit at fixed offsets from it.  Each thread owns one column:
// the 2K+1 x-band coefficients of the column and the RROWS+2K values of x down the column sit in
// registers, so the y-sums of all RROWS rows come from that window, and only the x-neighbours
// are read from LDS, as are the y-band coefficients, M_y and the Dirichlet flags of the
// work-group's rows (staged with x).  b of the column's rows is requested before the staging, so
// its latency overlaps it.  Needs Nx <= 256 (one column per thread).  res_rows leaves the result
// of row rl, column ix to out(rl, iy, ix, value, b, x) (b and x of a free node, 0 on Dirichlet
// nodes and for apply_only, for the convergence test); the LDS it uses is res_rows_lds(Nx)
// doubles from xs.
#define RROWS 16
__host__ __device__ constexpr long res_rows_lds(int K, int Nx) {
  return (long)(RROWS + 2 * K) * (Nx + 2 * K) + RROWS * (2 * K + 3);
}

template <int K, class Out>
__device__ __forceinline__ void res_rows(const VGrid& vg, int Nx, int Ny, int perx, const double* __restrict__ KxB,
                                         const double* __restrict__ Mx, const unsigned char* __restrict__ dirx,
                                         const double* __restrict__ KyB, const double* __restrict__ My,
                                         const unsigned char* __restrict__ diry, const double* __restrict__ shift,
                                         const double* __restrict__ bb, const double* __restrict__ x, int apply_only,
                                         const unsigned char* __restrict__ ebot, double* xs, Out out) {
  constexpr int NB = 2 * K + 1, NW = RROWS + 2 * K;
  const int LR = Nx + 2 * K;        // staged row: x[iy][ix] at K + ix
  double* kyl = xs + NW * LR;       // [RROWS][NB] y-band rows iy0..
  double* myl = kyl + RROWS * NB;   // [RROWS] M_y
  double* dyl = myl + RROWS;        // [RROWS] Dirichlet flag of the row
  int rb, pl;
  xcd_tile(vg, rb, pl);
  const int iy0 = rb * RROWS;
  const long Ng = (long)Nx * Ny;
  const double* xp = x + pl * Ng;
  const int ix = threadIdx.x, ixc = ix < Nx ? ix : Nx - 1;   // threads past Nx load column Nx - 1
  double bv[RROWS];
  if (!apply_only) {
#pragma unroll
    for (int rl = 0; rl < RROWS; ++rl) bv[rl] = bb[pl * Ng + (long)min(iy0 + rl, Ny - 1) * Nx + ixc];
  }
  stage_lds<256, 16, double>(
      NW * LR,
      [&](int idx) {
        const int rr = idx / LR;
        int jx = idx - rr * LR - K;
        const bool in = jx >= 0 && jx < Nx;
        if (perx) jx = jx < 0 ? jx + Nx : (jx >= Nx ? jx - Nx : jx);
        const int iy = iy0 - K + rr;
        const bool ok = iy >= 0 && iy < Ny && (in || perx);
        const double v = xp[(long)(ok ? iy : 0) * Nx + (ok ? jx : 0)];
        return ok ? v : 0.0;
      },
      [&](int idx, double v) { xs[idx] = v; });
  for (int idx = threadIdx.x; idx < RROWS * (NB + 2); idx += 256) {   // <= 2 rounds
    const int rl = idx % RROWS, q = idx / RROWS;
    const int iy = min(iy0 + rl, Ny - 1);
    if (q < NB) kyl[rl * NB + q] = KyB[(long)q * Ny + iy];
    else if (q == NB) myl[rl] = My[iy];
    else dyl[rl] = diry[iy] ? 1.0 : 0.0;
  }
  double kx[NB];
#pragma unroll
  for (int d = 0; d < NB; ++d) kx[d] = KxB[(long)d * Nx + ixc];
  const double mx = Mx[ixc], sh = shift[pl];
  const bool dxn = dirx[ixc] != 0;
  const bool egap = ebot && !ebot[ixc];   // bottom-row gap node of a partial electrode set
  __syncthreads();
  if (ix >= Nx) return;
  const int rend = min(RROWS, Ny - iy0);
  double win[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) win[q] = xs[q * LR + K + ix];
#pragma unroll
  for (int rl = 0; rl < RROWS; ++rl) {
    if (rl < rend) {
      const int iy = iy0 + rl;
      const double* row = xs + (rl + K) * LR + ix;   // x[iy][ix + d - K] at row[d]
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int d = 0; d < NB; ++d) ax += kx[d] * row[d];
#pragma unroll
      for (int d = 0; d < NB; ++d) ay += kyl[rl * NB + d] * win[rl + d];
      const double xv = win[rl + K];
      const double my = myl[rl];
      const double Av = ax * my + mx * ay + sh * mx * my * xv;
      if (apply_only) {
        out(rl, iy, ix, Av, 0.0, 0.0);
      } else {
        // is_dir: x-Dirichlet column, or a y-Dirichlet row except the gap nodes of the bottom row
        const bool dn = dxn || (dyl[rl] != 0.0 && !(iy == 0 && egap));
        out(rl, iy, ix, dn ? 0.0 : bv[rl] - Av, dn ? 0.0 : bv[rl], dn ? 0.0 : xv);
      }
    }
  }
}

template <int K>
__device__ __forceinline__ void k_residual_lds_run(const VGrid& vg, int Nx, int Ny, int perx,
                                                   const double* __restrict__ KxB, const double* __restrict__ Mx,
                                                   const unsigned char* __restrict__ dirx,
                                                   const double* __restrict__ KyB, const double* __restrict__ My,
                                                   const unsigned char* __restrict__ diry,
                                                   const double* __restrict__ shift, const double* __restrict__ bb,
                                                   const double* __restrict__ x, double* __restrict__ r,
                                                   int apply_only, const unsigned char* __restrict__ ebot, Chk ck) {
  if (ck.gin && *ck.gin) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xs = reinterpret_cast<double*>(smem_raw);
  int rb, pl;
  xcd_tile(vg, rb, pl);   // the tile res_rows takes
  const long Ng = (long)Nx * Ny, pofs = (long)pl * Ng;
  double r2 = 0.0, x2 = 0.0;
  res_rows<K>(vg, Nx, Ny, perx, KxB, Mx, dirx, KyB, My, diry, shift, bb, x, apply_only, ebot, xs,
              [&](int, int iy, int ix, double v, double bv, double xv) {
                r[pofs + (long)iy * Nx + ix] = v;
                r2 += v * v;
                x2 += xv * xv;
              });
  if (ck.part) {
    const double an = ck.anorm[pl % ck.nplane];
    chk_store(vg, ck, r2, an * an * x2);
  }
}
template <int K>
struct k_residual_lds : KDef<&k_residual_lds_run<K>, 256, 0> {};

// Batched GEMM on the matrix cores for the fast-diagonalisation passes:
//   C[p] (M x N) = A[p] (M x K) * B[p] (K x N), row-major, plane strides sA, sB (0: shared).
// One work-group (four waves) computes one 16x16 output tile with v_mfma_{f64,f32}_16x16x4
// (operands straight from L2 into the MFMA register layout).  Within each 16-wide slice of K, lane
// group g = lane/16 takes k = k0 + 4g + s at MFMA step s (s = 0..3): a permutation of the
// contraction index applied to both operands, which makes each lane's A reads contiguous.
// The next slice is loaded while the current one is multiplied.  Epilogues:
//   EPI 0: C = acc
//   EPI 1: C = acc / (lr[m] + lc[n] + shift[p])   (0 where the denominator vanishes: the
//          constant null mode of a singular operator)
//   EPI 2: X += acc   (FP64 accumulation of the correction)
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double V __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element j of lane group g holds row 4j + g (measured on gfx950)
  static __device__ __forceinline__ int row(int g, int j) { return 4 * j + g; }
};
template <>
struct Mfma<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element j of lane group g holds row 4g + j
  static __device__ __forceinline__ int row(int g, int j) { return 4 * g + j; }
};

template <typename T, typename TA, typename TB, int EPI>
__device__ __forceinline__ void k_gemm_run(const VGrid& vg, const TA* __restrict__ A, long sA,
                                           const TB* __restrict__ B, long sB, int M, int N, int K, T* __restrict__ C,
                                           long sC, const double* __restrict__ lr, const double* __restrict__ lc,
                                           const double* __restrict__ shift, double* __restrict__ X,
                                           const TB* __restrict__ B2, double cb1, double cb2,
                                           const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  // B2 != nullptr: the right operand is cb1 B + cb2 B2 (e.g. the BDF extrapolation of a field)
  // four waves split K: wave w takes the 16-wide slices w, w+4, w+8, ... of the contraction,
  // and the partial tiles are summed in LDS in a fixed order (deterministic)
  __shared__ T red[4][4][64];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int n0 = vg.b.x * 16, m0 = vg.b.y * 16, pl = vg.b.z;
  const int m = m0 + r16, n = n0 + r16;
  const bool mok = m < M, nok = n < N;
  const TA* Arow = A + pl * sA + (long)(mok ? m : 0) * K;
  const TB* Bcol = B + pl * sB + (nok ? n : 0);
  const TB* B2col = B2 ? B2 + pl * sB + (nok ? n : 0) : nullptr;
  auto ldb = [&](long o) -> T { return B2col ? T(cb1 * double(Bcol[o]) + cb2 * double(B2col[o])) : T(Bcol[o]); };
  typename Mfma<T>::V acc = {T(0), T(0), T(0), T(0)};
  T a[4], b[4], an[4], bn[4];
  const int kstart = 16 * w;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = kstart + 4 * g + s;
    const int kk = k < K ? k : K - 1;
    a[s] = T(Arow[kk]);
    b[s] = ldb((long)kk * N);
  }
  for (int k0 = kstart; k0 < K; k0 += 64) {
    const int k1 = k0 + 64;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k1 + 4 * g + s;
      const int kk = k < K ? k : K - 1;
      an[s] = T(Arow[kk]);
      bn[s] = ldb((long)kk * N);
    }
    // loads are clamped in range and left unmasked (rows >= M and columns >= N are never
    // stored); contraction indices >= K occur only in the last slice and are zeroed there
    if (k0 + 16 <= K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = Mfma<T>::op(a[s], b[s], acc);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = Mfma<T>::op((k0 + 4 * g + s < K) ? a[s] : T(0), b[s], acc);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[s] = an[s];
      b[s] = bn[s];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) red[w][j][lane] = acc[j];
  __syncthreads();
  if (w != 0) return;
  // accumulator layout: lane (g, r16) holds column r16 of four rows (Mfma<T>::row)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const T v = ((red[0][j][lane] + red[1][j][lane]) + red[2][j][lane]) + red[3][j][lane];
    const int mm = m0 + Mfma<T>::row(g, j);
    if (mm >= M || !nok) continue;
    const long o = pl * sC + (long)mm * N + n;
    if (EPI == 0) {
      C[o] = v;
    } else if (EPI == 1) {
      const double den = lr[mm] + lc[n] + shift[pl];
      C[o] = (den != 0.0) ? T(double(v) / den) : T(0);
    } else if (EPI == 2) {
      X[o] += double(v);
    } else {
      X[o] = double(v);
    }
  }
}
template <typename T, typename TA, typename TB, int EPI>
struct k_gemm : KDef<&k_gemm_run<T, TA, TB, EPI>, 256, 0> {};

// Register-blocked batched GEMM (same operands, layout and epilogues as k_gemm): one wave
// computes a (16 TM) x (16 TN) block of C with TM*TN accumulator tiles, so each loaded A
// fragment feeds TN and each B fragment TM matrix-core ops; the SK waves of a work-group take
// the 16-wide contraction slices w, w+SK, ... and their partial blocks are summed through LDS
// in a fixed order.  The next slice's fragments are loaded while the current one is multiplied.
template <typename T, typename TA, typename TB, int EPI, int TM, int TN, int SK>
__device__ __forceinline__ void k_gemmt_run(const VGrid& vg, const TA* __restrict__ A, long sA,
                                            const TB* __restrict__ B, long sB, int M, int N, int K, T* __restrict__ C,
                                            long sC, const double* __restrict__ lr, const double* __restrict__ lc,
                                            const double* __restrict__ shift, double* __restrict__ X,
                                            const TB* __restrict__ B2, double cb1, double cb2,
                                            const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef typename Mfma<T>::V V;
  constexpr int NR = SK > 1 ? SK - 1 : 1;
  __shared__ T red[NR][TM * TN * 4][64];
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int n0 = vg.b.x * 16 * TN, m0 = vg.b.y * 16 * TM, pl = vg.b.z;
  const TA* Ap = A + pl * sA;
  const TB* Bp = B + pl * sB;
  const TB* B2p = B2 ? B2 + pl * sB : nullptr;
  long arow[TM];
  int bcol[TN];
  bool mok[TM], nok[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int m = m0 + 16 * i + r16;
    mok[i] = m < M;
    arow[i] = (long)(mok[i] ? m : 0) * K;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + 16 * j + r16;
    nok[j] = n < N;
    bcol[j] = nok[j] ? n : 0;
  }
  V acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = V{T(0), T(0), T(0), T(0)};
  T a[TM][4], b[TN][4];
  auto load = [&](int k0, T (&aa)[TM][4], T (&bb)[TN][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const bool kok = k < K;
      const int kk = kok ? k : 0;
#pragma unroll
      for (int i = 0; i < TM; ++i) aa[i][s] = T(Ap[arow[i] + kk]);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const long o = (long)kk * N + bcol[j];
        bb[j][s] = B2p ? T(cb1 * double(Bp[o]) + cb2 * double(B2p[o])) : T(Bp[o]);
      }
    }
  };
  const int kstep = 16 * SK;
  if (16 * w < K) load(16 * w, a, b);
  for (int k0 = 16 * w; k0 < K; k0 += kstep) {
    T an[TM][4], bn[TN][4];
    if (k0 + kstep < K) load(k0 + kstep, an, bn);
    if (k0 + 16 <= K) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::op(a[i][s], b[j][s], acc[i][j]);
    } else {   // last, partial slice: zero the contraction indices >= K
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool kok = k0 + 4 * g + s < K;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<T>::op(kok ? a[i][s] : T(0), b[j][s], acc[i][j]);
      }
    }
    if (k0 + kstep < K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i][s] = an[i][s];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j][s] = bn[j][s];
      }
    }
  }
  if (SK > 1) {
    if (w > 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) red[w - 1][(i * TN + j) * 4 + q][lane] = acc[i][j][q];
    }
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          T v = acc[i][j][q];
#pragma unroll
          for (int r = 0; r < SK - 1; ++r) v += red[r][(i * TN + j) * 4 + q][lane];
          acc[i][j][q] = v;
        }
  }
  // accumulator layout: lane (g, r16) holds column r16 of four rows (Mfma<T>::row) of each tile
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + 16 * j + r16;
      if (n >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int mm = m0 + 16 * i + Mfma<T>::row(g, q);
        if (mm >= M) continue;
        const T v = acc[i][j][q];
        const long o = pl * sC + (long)mm * N + n;
        if (EPI == 0) {
          C[o] = v;
        } else if (EPI == 1) {
          const double den = lr[mm] + lc[n] + shift[pl];
          C[o] = (den != 0.0) ? T(double(v) / den) : T(0);
        } else if (EPI == 2) {
          X[o] += double(v);
        } else {
          X[o] = double(v);
        }
      }
    }
}
template <typename T, typename TA, typename TB, int EPI, int TM, int TN, int SK>
struct k_gemmt : KDef<&k_gemmt_run<T, TA, TB, EPI, TM, TN, SK>, 64 * SK, 0> {};

// Small-operand-in-LDS batched GEMMs.  In every product of the solves and z transforms one
// operand is a small shared matrix S (a 1D eigenvector matrix or a DFT matrix, <= 320^2) and the
// other streams the field planes.  The work-group copies the slice of S it needs into LDS once
// and streams the plane operand from HBM exactly once, with the contraction split into chunks of
// four 16-wide slices whose loads are issued one chunk ahead.  The streamed dimension is
// flattened over planes, so nothing is padded per plane.
//   k_gemm_sr:  C (P*M x N) = A (P*M x K, streamed rows) * S (K x N)           [S right]
//   k_gemm_sl:  C_p (M x N) = S (M x K) * B_p (K x N), columns (p, n) flattened [S left]
// A work-group has four waves: 4/SK of them take 16-wide tiles of the streamed dimension and
// SK split the contraction (partials summed through LDS in a fixed order); each wave holds W
// accumulator tiles along the small dimension (16 W wide).  Epilogues as k_gemm.
#define GEMM_CHUNK 4

template <typename T, typename TA, int EPI, int W, int SK>
__device__ __forceinline__ void k_gemm_sr_run(const VGrid& vg, const TA* __restrict__ A, const T* __restrict__ S,
                                              int Mtot, int N, int K, T* __restrict__ C, double* __restrict__ X,
                                              const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef typename Mfma<T>::V V;
  constexpr int WS = 4 / SK, NP = 16 * W + 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Sl = reinterpret_cast<T*>(smem_raw);
  const int KP = (K + 15) & ~15;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  int tbx, tby;
  xcd_tile_yfast(vg, tbx, tby);   // row tile tbx, column block tby
  const int n0 = tby * 16 * W;
  const int ms = w % WS, ks = w / WS;
  const int m = (tbx * WS + ms) * 16 + r16;
  const bool mok = m < Mtot;
  const TA* Am = A + (long)(mok ? m : 0) * K;
  V acc[W];
#pragma unroll
  for (int j = 0; j < W; ++j) acc[j] = V{T(0), T(0), T(0), T(0)};
  const int nsl = KP / 16;                       // 16-wide slices; this wave takes ks, ks+SK, ...
  const int nsw = nsl > ks ? (nsl - ks + SK - 1) / SK : 0;
  const int nfull = nsw / GEMM_CHUNK, rem = nsw - nfull * GEMM_CHUNK;
  T a[GEMM_CHUNK][4], an[GEMM_CHUNK][4];
  // loads past the wave's last slice are clamped in range and never multiplied
  auto load = [&](int c0, T (&aa)[GEMM_CHUNK][4]) {
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q) {
      const int sl = ks + SK * (c0 + q);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 16 * sl + 4 * g + s;
        aa[q][s] = T(Am[k < K ? k : K - 1]);   // S rows >= K are zero in LDS
      }
    }
  };
  auto mma = [&](int sl, const T (&av)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T* Srow = Sl + (16 * sl + 4 * g + s) * NP + r16;
#pragma unroll
      for (int j = 0; j < W; ++j) acc[j] = Mfma<T>::op(av[s], Srow[16 * j], acc[j]);
    }
  };
  load(0, a);   // the first chunk of A is in flight while S is staged
  // S[k][n0 .. n0+16W) -> LDS (zero beyond K or N)
  stage_lds<256, 16, T>(
      KP * 16 * W,
      [&](int idx) {
        const int k = idx / (16 * W), j = idx - k * (16 * W);
        const int n = n0 + j;
        const bool ok = k < K && n < N;
        const T v = S[(long)(k < K ? k : K - 1) * N + (n < N ? n : N - 1)];
        return ok ? v : T(0);
      },
      [&](int idx, T v) {
        const int k = idx / (16 * W), j = idx - k * (16 * W);
        Sl[k * NP + j] = v;
      });
  __syncthreads();
  for (int ch = 0; ch < nfull; ++ch) {
    load((ch + 1) * GEMM_CHUNK, an);
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q) mma(ks + SK * (ch * GEMM_CHUNK + q), a[q]);
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) a[q][s] = an[q][s];
  }
#pragma unroll
  for (int q = 0; q < GEMM_CHUNK - 1; ++q)
    if (q < rem) mma(ks + SK * (nfull * GEMM_CHUNK + q), a[q]);
  if (SK > 1) {
    T* red = Sl + KP * NP;   // [SK-1][WS][W*4][64]
    __syncthreads();
    if (ks > 0) {
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(((ks - 1) * WS + ms) * W * 4 + j * 4 + q) * 64 + lane] = acc[j][q];
    }
    __syncthreads();
    if (ks != 0) return;
#pragma unroll
    for (int j = 0; j < W; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T v = acc[j][q];
        for (int r = 0; r < SK - 1; ++r) v += red[((r * WS + ms) * W * 4 + j * 4 + q) * 64 + lane];
        acc[j][q] = v;
      }
  }
  const int mb = (tbx * WS + ms) * 16;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const int n = n0 + 16 * j + r16;
    if (n >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int mm = mb + Mfma<T>::row(g, q);
      if (mm >= Mtot) continue;
      const long o = (long)mm * N + n;
      if (EPI == 0)
        C[o] = acc[j][q];
      else if (EPI == 2)
        X[o] += double(acc[j][q]);
      else
        X[o] = double(acc[j][q]);
    }
  }
}
template <typename T, typename TA, int EPI, int W, int SK>
struct k_gemm_sr : KDef<&k_gemm_sr_run<T, TA, EPI, W, SK>, 256, 0> {};

template <typename T, typename TB, int EPI, int W, int SK>
__device__ __forceinline__ void k_gemm_sl_run(const VGrid& vg, const T* __restrict__ S, const TB* __restrict__ B,
                                              long sB, int planes, int M, int N, int K, T* __restrict__ C, long sC,
                                              const double* __restrict__ lr, const double* __restrict__ lc,
                                              const double* __restrict__ shift, const TB* __restrict__ B2, double cb1,
                                              double cb2, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef typename Mfma<T>::V V;
  constexpr int WS = 4 / SK, MP = 16 * W + 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Sl = reinterpret_cast<T*>(smem_raw);    // [k][i - m0] = S[i][k]
  const int KP = (K + 15) & ~15;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  int tbx, tby;
  xcd_tile_yfast(vg, tbx, tby);   // column tile tbx, row block tby
  const int m0 = tby * 16 * W;
  const int ms = w % WS, ks = w / WS;
  const long ctot = (long)planes * N;
  const long cidx = ((long)tbx * WS + ms) * 16 + r16;
  const bool cok = cidx < ctot;
  const int p = cok ? (int)(cidx / N) : 0;
  const int n = cok ? (int)(cidx - (long)p * N) : 0;
  const TB* Bp = B + p * sB + n;
  const TB* B2p = B2 ? B2 + p * sB + n : nullptr;
  V acc[W];
#pragma unroll
  for (int j = 0; j < W; ++j) acc[j] = V{T(0), T(0), T(0), T(0)};
  const int nsl = KP / 16;
  const int nsw = nsl > ks ? (nsl - ks + SK - 1) / SK : 0;
  const int nfull = nsw / GEMM_CHUNK, rem = nsw - nfull * GEMM_CHUNK;
  T b[GEMM_CHUNK][4], bn[GEMM_CHUNK][4], b2[GEMM_CHUNK][4], b2n[GEMM_CHUNK][4];
  // loads past the wave's last slice are clamped in range and never multiplied; the
  // two-source combination is formed when the values are consumed
  auto load = [&](int c0, T (&bb)[GEMM_CHUNK][4], T (&bb2)[GEMM_CHUNK][4]) {
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q) {
      const int sl = ks + SK * (c0 + q);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 16 * sl + 4 * g + s;
        const long o = (long)(k < K ? k : K - 1) * N;   // S^T rows >= K are zero in LDS
        bb[q][s] = T(Bp[o]);
        if (B2p) bb2[q][s] = T(B2p[o]);
      }
    }
  };
  auto mma = [&](int sl, const T (&bv)[4], const T (&bv2)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const T x = B2p ? T(cb1 * double(bv[s]) + cb2 * double(bv2[s])) : bv[s];
      const T* Srow = Sl + (16 * sl + 4 * g + s) * MP + r16;
#pragma unroll
      for (int t = 0; t < W; ++t) acc[t] = Mfma<T>::op(Srow[16 * t], x, acc[t]);
    }
  };
  load(0, b, b2);   // the first chunk of B is in flight while S is staged
  stage_lds<256, 16, T>(
      16 * W * KP,
      [&](int idx) {
        const int i = idx / KP, k = idx - i * KP;
        const int mi = m0 + i;
        const bool ok = k < K && mi < M;
        const T v = S[(long)(mi < M ? mi : M - 1) * K + (k < K ? k : K - 1)];
        return ok ? v : T(0);
      },
      [&](int idx, T v) {
        const int i = idx / KP, k = idx - i * KP;
        Sl[k * MP + i] = v;
      });
  __syncthreads();
  for (int ch = 0; ch < nfull; ++ch) {
    load((ch + 1) * GEMM_CHUNK, bn, b2n);
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q) mma(ks + SK * (ch * GEMM_CHUNK + q), b[q], b2[q]);
#pragma unroll
    for (int q = 0; q < GEMM_CHUNK; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        b[q][s] = bn[q][s];
        b2[q][s] = b2n[q][s];
      }
  }
#pragma unroll
  for (int q = 0; q < GEMM_CHUNK - 1; ++q)
    if (q < rem) mma(ks + SK * (nfull * GEMM_CHUNK + q), b[q], b2[q]);
  if (SK > 1) {
    T* red = Sl + KP * MP;
    __syncthreads();
    if (ks > 0) {
#pragma unroll
      for (int t = 0; t < W; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[(((ks - 1) * WS + ms) * W * 4 + t * 4 + q) * 64 + lane] = acc[t][q];
    }
    __syncthreads();
    if (ks != 0) return;
#pragma unroll
    for (int t = 0; t < W; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T v = acc[t][q];
        for (int r = 0; r < SK - 1; ++r) v += red[((r * WS + ms) * W * 4 + t * 4 + q) * 64 + lane];
        acc[t][q] = v;
      }
  }
  if (!cok) return;
  T* Cp = C + p * sC + n;
#pragma unroll
  for (int t = 0; t < W; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = m0 + 16 * t + Mfma<T>::row(g, q);
      if (i >= M) continue;
      if (EPI == 0) {
        Cp[(long)i * N] = acc[t][q];
      } else {
        const double den = lr[i] + lc[n] + shift[p];
        Cp[(long)i * N] = (den != 0.0) ? T(double(acc[t][q]) / den) : T(0);
      }
    }
}
template <typename T, typename TB, int EPI, int W, int SK>
struct k_gemm_sl : KDef<&k_gemm_sl_run<T, TB, EPI, W, SK>, 256, 0> {};

// Configurations the autotuner chooses from.  0..7: register-blocked k_gemm / k_gemmt tiles
// {TM, TN, SK} (entry 0 is k_gemm: 16 x 16 tile, four-wave split K); 8..15: the LDS kernels
// k_gemm_sr / k_gemm_sl {W, SK} (used where one operand is shared by all planes and fits).
struct GemmCfg {
  int tm, tn, sk;
};
static const GemmCfg kGemmCfg[8] = {{1, 1, 4}, {2, 2, 1}, {2, 2, 2}, {3, 3, 1},
                                    {3, 3, 2}, {2, 4, 1}, {4, 2, 1}, {2, 2, 4}};
static const GemmCfg kLdsCfg[8] = {{1, 1, 0}, {2, 1, 0}, {3, 1, 0}, {1, 2, 0},
                                   {2, 2, 0}, {3, 2, 0}, {1, 4, 0}, {2, 4, 0}};
#define GEMM_LDS_MAX (64 * 1024)

template <typename T, typename TA, typename TB, int EPI>
static bool gemm_launch(pfd_ctx* c, int cfg, int cls, int planes, const TA* A, long sA, const TB* B, long sB,
                        int M, int N, int K, T* C, long sC, const double* lr, const double* lc,
                        const double* shift, double* X, const TB* B2, double cb1, double cb2) {
  ProfScope ps(c, cls);
  if (cfg >= 8) {
    const int W = kLdsCfg[cfg - 8].tm, SK = kLdsCfg[cfg - 8].tn, WS = 4 / SK;
    const long KP = (K + 15) & ~15;
    const size_t lds = sizeof(T) * (KP * (16 * W + 4) + (SK > 1 ? (long)(SK - 1) * WS * W * 4 * 64 : 0));
    const bool sr = (sB == 0 && B2 == nullptr && EPI != 1 && (planes == 1 || (sA == (long)M * K && sC == (long)M * N)));
    const bool sl = (sA == 0 && (EPI == 0 || EPI == 1));
    if (lds > GEMM_LDS_MAX || (!sr && !sl)) return false;
    if (sr) {
      if constexpr (EPI != 1 && std::is_same<TB, T>::value) {
        const int Mtot = planes * M;
        dim3 grid((Mtot + 16 * WS - 1) / (16 * WS), (N + 16 * W - 1) / (16 * W));
#define SR_CASE(W_, SK_)                                                                                   \
  if (W == W_ && SK == SK_)                                                                                \
    Kern<k_gemm_sr<T, TA, EPI, W_, SK_>>::launch(c, -1, grid, dim3(256), lds, c->stream, A, (const T*)B, Mtot, N, \
                       K, C, X, c->gate);
        SR_CASE(1, 1) SR_CASE(2, 1) SR_CASE(3, 1) SR_CASE(1, 2) SR_CASE(2, 2) SR_CASE(3, 2) SR_CASE(1, 4)
        SR_CASE(2, 4)
#undef SR_CASE
        return true;
      }
      return false;
    }
    if constexpr ((EPI == 0 || EPI == 1) && std::is_same<TA, T>::value) {
      const long ctot = (long)planes * N;
      dim3 grid((unsigned)((ctot + 16 * WS - 1) / (16 * WS)), (M + 16 * W - 1) / (16 * W));
#define SL_CASE(W_, SK_)                                                                                   \
  if (W == W_ && SK == SK_)                                                                                \
    Kern<k_gemm_sl<T, TB, EPI, W_, SK_>>::launch(c, -1, grid, dim3(256), lds, c->stream, (const T*)A, B, sB,     \
                       planes, M, N, K, C, sC, lr, lc, shift, B2, cb1, cb2, c->gate);
      SL_CASE(1, 1) SL_CASE(2, 1) SL_CASE(3, 1) SL_CASE(1, 2) SL_CASE(2, 2) SL_CASE(3, 2) SL_CASE(1, 4)
      SL_CASE(2, 4)
#undef SL_CASE
      return true;
    }
    return false;
  }
  const GemmCfg& q = kGemmCfg[cfg];
  dim3 grid((N + 16 * q.tn - 1) / (16 * q.tn), (M + 16 * q.tm - 1) / (16 * q.tm), planes);
#define GEMMT_CASE(ID, TM_, TN_, SK_)                                                                  \
  case ID:                                                                                             \
    Kern<k_gemmt<T, TA, TB, EPI, TM_, TN_, SK_>>::launch(c, -1, grid, dim3(64 * SK_), 0, c->stream, A, sA, B, \
                       sB, M, N, K, C, sC, lr, lc, shift, X, B2, cb1, cb2, c->gate);                   \
    break;
  switch (cfg) {
    case 0:
      Kern<k_gemm<T, TA, TB, EPI>>::launch(c, -1, grid, dim3(256), 0, c->stream, A, sA, B, sB, M, N, K, C, sC, lr,
                         lc, shift, X, B2, cb1, cb2, c->gate);
      break;
    GEMMT_CASE(1, 2, 2, 1)
    GEMMT_CASE(2, 2, 2, 2)
    GEMMT_CASE(3, 3, 3, 1)
    GEMMT_CASE(4, 3, 3, 2)
    GEMMT_CASE(5, 2, 4, 1)
    GEMMT_CASE(6, 4, 2, 1)
    GEMMT_CASE(7, 2, 2, 4)
    default:
      return false;
  }
#undef GEMMT_CASE
  return true;
}

template <typename T, typename TA, typename TB, int EPI>
static void gemm(pfd_ctx* c, int site, int planes, const TA* A, long sA, const TB* B, long sB, int M, int N, int K,
                 T* C, long sC, const double* lr, const double* lc, const double* shift, double* X) {
  const int cls = sizeof(T) == 8 ? PFD_PROF_GEMM64 : PFD_PROF_GEMM32;
  if (!gemm_launch<T, TA, TB, EPI>(c, c->gemm_cfg[site][sizeof(T) == 8 ? 1 : 0], cls, planes, A, sA, B, sB, M, N,
                                   K, C, sC, lr, lc, shift, X, (const TB*)nullptr, 1.0, 0.0))
    gemm_launch<T, TA, TB, EPI>(c, 0, cls, planes, A, sA, B, sB, M, N, K, C, sC, lr, lc, shift, X,
                                (const TB*)nullptr, 1.0, 0.0);
}

// ------------------------------------------------------------------ fused fast diagonalisation
// One correction x (+)= Sy [ (Sy^T r Sx) ./ (ly (+) lx + shift) ] Sx^T in two launches instead of four
// GEMM passes, each work-group owning one 16-wide strip of one plane, so the intermediate strip
// stays in LDS:
//   k_fdm1, column strip cs:  u = r Sx[:, cs] (Ny x 16, LDS);  t[:, cs] = (Sy^T u) ./ den  -> t
//   k_fdm2, row strip rs:     v = Sy[rs, :] t (16 x Nx, LDS);  x[rs, :] (+)= v Sx^T
// Small shared operands (Sx, Sy and their transposes, <= 320^2) are read through L1/L2; the
// plane operands r, t are streamed once per strip.  MFMA 16x16x4 in the operand precision T
// with the contraction permutation k = k0 + 4g + s of k_gemm; the four waves of a work-group
// split the output tiles of each stage.  Work-groups of one plane are placed on one XCD (the
// hardware hands work-groups to the eight XCDs round robin) when the plane count allows, so
// the strips of a plane share that XCD's L2.
#define FDM_LDU 17                          // LDS row pitch of u (bank spread)
#define FDM_MAXT ((PFD_NMAX + 63) / 64)     // output tiles per wave (20 tiles over 4 waves)

__device__ __forceinline__ void fdm_map(const VGrid& vg, int nstrip, int planes, int& p, int& st) {
  const int L = vg.b.x;
  if ((planes & 7) == 0) {
    const int xcd = L & 7, idx = L >> 3;
    p = xcd + 8 * (idx / nstrip);
    st = idx % nstrip;
  } else {
    p = L / nstrip;
    st = L % nstrip;
  }
}

template <typename T>
__device__ __forceinline__ void k_fdm1_run(const VGrid& vg, int planes, int Ny, int Nx, long Ng,
                                           const double* __restrict__ r, const T* __restrict__ SxT,
                                           const T* __restrict__ SyT, const double* __restrict__ ly,
                                           const double* __restrict__ lx, const double* __restrict__ shift,
                                           T* __restrict__ t, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  __shared__ T u[PFD_NMAX * FDM_LDU];
  typedef typename Mfma<T>::V V;
  const int nstrip = (Nx + 15) >> 4, mtiles = (Ny + 15) >> 4;
  int p, cs;
  fdm_map(vg, nstrip, planes, p, cs);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), r16 = lane & 15, g = lane >> 4;
  const int n = cs * 16 + r16;
  const bool nok = n < Nx;
  const double* rp = r + (long)p * Ng;
  // ---- u = r Sx[:, strip]: tiles mt = w, w+4, ... over the Ny rows
  V acc[FDM_MAXT];
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) acc[i] = V{T(0), T(0), T(0), T(0)};
  const T* Bn = SxT + (long)(nok ? n : 0) * Nx;   // row n of Sx^T = column n of Sx
  for (int k0 = 0; k0 < Nx; k0 += 16) {
    T b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const T bv = Bn[k < Nx ? k : Nx - 1];
      b[s] = (nok && k < Nx) ? bv : T(0);
    }
#pragma unroll
    for (int i = 0; i < FDM_MAXT; ++i) {
      const int mt = w + 4 * i;
      if (mt >= mtiles) break;
      const int m = mt * 16 + r16;
      const double* Am = rp + (long)(m < Ny ? m : 0) * Nx;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        const T av = T(Am[k < Nx ? k : Nx - 1]);
        const T a = (m < Ny && k < Nx) ? av : T(0);
        acc[i] = Mfma<T>::op(a, b[s], acc[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) {
    const int mt = w + 4 * i;
    if (mt >= mtiles) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) u[(mt * 16 + Mfma<T>::row(g, j)) * FDM_LDU + r16] = acc[i][j];
  }
  __syncthreads();
  // ---- t[:, strip] = (Sy^T u) ./ den: tiles over the Ny rows again; u rows >= Ny are zero
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) acc[i] = V{T(0), T(0), T(0), T(0)};
  const int K2 = mtiles * 16;
  for (int k0 = 0; k0 < K2; k0 += 16) {
    T b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) b[s] = u[(k0 + 4 * g + s) * FDM_LDU + r16];
#pragma unroll
    for (int i = 0; i < FDM_MAXT; ++i) {
      const int at = w + 4 * i;
      if (at >= mtiles) break;
      const int a = at * 16 + r16;
      const T* Aa = SyT + (long)(a < Ny ? a : 0) * Ny;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        const T aw = Aa[k < Ny ? k : Ny - 1];
        const T av = (a < Ny && k < Ny) ? aw : T(0);
        acc[i] = Mfma<T>::op(av, b[s], acc[i]);
      }
    }
  }
  if (!nok) return;
  const double lcol = lx[n] + shift[p];
  T* tp = t + (long)p * Ng;
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) {
    const int at = w + 4 * i;
    if (at >= mtiles) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = at * 16 + Mfma<T>::row(g, j);
      if (a >= Ny) continue;
      const double den = ly[a] + lcol;
      tp[(long)a * Nx + n] = (den != 0.0) ? T(double(acc[i][j]) / den) : T(0);
    }
  }
}
template <typename T>
struct k_fdm1 : KDef<&k_fdm1_run<T>, 256, 0> {};

template <typename T, bool OVERWRITE>
__device__ __forceinline__ void k_fdm2_run(const VGrid& vg, int planes, int Ny, int Nx, long Ng,
                                           const T* __restrict__ t, const T* __restrict__ Sy,
                                           const T* __restrict__ Sx, double* __restrict__ x,
                                           const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  __shared__ T v[16 * (PFD_NMAX + 1)];
  typedef typename Mfma<T>::V V;
  const int nstrip = (Ny + 15) >> 4, ntiles = (Nx + 15) >> 4;
  const int ldv = ntiles * 16 + 1;
  int p, rs;
  fdm_map(vg, nstrip, planes, p, rs);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), r16 = lane & 15, g = lane >> 4;
  const T* tp = t + (long)p * Ng;
  // ---- v = Sy[strip, :] t: A operand row i = rs*16 + r16 of Sy (shared by the wave's tiles)
  const int ia = rs * 16 + r16;
  const bool iok = ia < Ny;
  const T* Ai = Sy + (long)(iok ? ia : 0) * Ny;
  V acc[FDM_MAXT];
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) acc[i] = V{T(0), T(0), T(0), T(0)};
  for (int k0 = 0; k0 < Ny; k0 += 16) {
    T a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const T av = Ai[k < Ny ? k : Ny - 1];
      a[s] = (iok && k < Ny) ? av : T(0);
    }
#pragma unroll
    for (int i = 0; i < FDM_MAXT; ++i) {
      const int nt = w + 4 * i;
      if (nt >= ntiles) break;
      const int n = nt * 16 + r16;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        const T bv = tp[(long)(k < Ny ? k : Ny - 1) * Nx + (n < Nx ? n : Nx - 1)];
        const T b = (n < Nx && k < Ny) ? bv : T(0);
        acc[i] = Mfma<T>::op(a[s], b, acc[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) {
    const int nt = w + 4 * i;
    if (nt >= ntiles) break;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[Mfma<T>::row(g, j) * ldv + nt * 16 + r16] = acc[i][j];
  }
  __syncthreads();
  // ---- x[strip, :] (+)= v Sx^T: B operand (k, n) = Sx[n][k]; v columns >= Nx are zero
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) acc[i] = V{T(0), T(0), T(0), T(0)};
  const int K2 = ntiles * 16;
  for (int k0 = 0; k0 < K2; k0 += 16) {
    T a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = v[r16 * ldv + k0 + 4 * g + s];
#pragma unroll
    for (int i = 0; i < FDM_MAXT; ++i) {
      const int nt = w + 4 * i;
      if (nt >= ntiles) break;
      const int n = nt * 16 + r16;
      const T* Bn = Sx + (long)(n < Nx ? n : 0) * Nx;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        const T bv = Bn[k < Nx ? k : Nx - 1];
        const T b = (n < Nx && k < Nx) ? bv : T(0);
        acc[i] = Mfma<T>::op(a[s], b, acc[i]);
      }
    }
  }
  double* xp = x + (long)p * Ng;
#pragma unroll
  for (int i = 0; i < FDM_MAXT; ++i) {
    const int nt = w + 4 * i;
    if (nt >= ntiles) break;
    const int n = nt * 16 + r16;
    if (n >= Nx) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rs * 16 + Mfma<T>::row(g, j);
      if (row >= Ny) continue;
      const long o = (long)row * Nx + n;
      if (OVERWRITE)
        xp[o] = double(acc[i][j]);
      else
        xp[o] += double(acc[i][j]);
    }
  }
}
template <typename T, bool OVERWRITE>
struct k_fdm2 : KDef<&k_fdm2_run<T, OVERWRITE>, 256, 0> {};

// Deterministic per-plane sums: part[p*PCH + blk] = sum over chunk blk of w_i f_i
// (w = M when weighted, else 1), for planes whose shift is 0 (singular operators).
// k_plane_sub then subtracts, per plane:
//   mode 0 (gauge int_h f = 0):    f -= (sum M f)/(sum M)
//   mode 1 (range projection):     f -= (sum f)/(sum M) * M
#define PCH 32
__device__ __forceinline__ void k_plane_sums_run(const VGrid& vg, long Ng, const double* __restrict__ Mdiag,
                                                 const double* __restrict__ shift, const double* __restrict__ f,
                                                 int weighted, double* __restrict__ part,
                                                 const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  const int blk = vg.b.x, pl = vg.b.y;
  __shared__ double sm[WG];
  double a = 0.0;
  if (shift[pl] == 0.0) {
    const long chunk = (Ng + PCH - 1) / PCH;
    const long i0 = blk * chunk, i1 = min(Ng, i0 + chunk);
    const double* fp = f + pl * Ng;
    for (long i = i0 + threadIdx.x; i < i1; i += WG) a += weighted ? Mdiag[i] * fp[i] : fp[i];
  }
  sm[threadIdx.x] = a;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[pl * PCH + blk] = sm[0];
}
struct k_plane_sums : KDef<&k_plane_sums_run, 0, 0> {};

__device__ __forceinline__ void k_plane_sub_run(const VGrid& vg, long Ng, int planes,
                                                const double* __restrict__ Mdiag, const double* __restrict__ shift,
                                                const double* __restrict__ part, double Mtot, int mode,
                                                double* __restrict__ f, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  const long id = (long)vg.b.x * blockDim.x + threadIdx.x;
  if (id >= planes * Ng) return;
  const int pl = (int)(id / Ng);
  if (shift[pl] != 0.0) return;
  double s = 0.0;
  for (int b = 0; b < PCH; ++b) s += part[pl * PCH + b];
  const long i = id - pl * Ng;
  f[id] -= (mode == 0) ? s / Mtot : s / Mtot * Mdiag[i];
}
struct k_plane_sub : KDef<&k_plane_sub_run, 0, 0> {};

static inline unsigned nblk(long n) { return (unsigned)((n + WG - 1) / WG); }


ProfScope::ProfScope(pfd_ctx* ctx, int k) : c(ctx), cls(k), i0(0), on(ctx && ctx->prof_on) {
  if (!on) return;
  if (c->ev_used + 2 > c->ev_pool.size()) {
    if (c->ev_pool.size() >= 200000) { on = false; return; }
    size_t n0 = c->ev_pool.size();
    c->ev_pool.resize(n0 + 4096);
    for (size_t i = n0; i < c->ev_pool.size(); ++i) (void)hipEventCreate(&c->ev_pool[i]);
  }
  i0 = c->ev_used;
  c->ev_used += 2;
  (void)hipEventRecord(c->ev_pool[i0], c->stream);
}

ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(c->ev_pool[i0 + 1], c->stream);
  c->prof_rec.push_back({cls, i0});
}

static void plane_fix(pfd_ctx* c, int fam, double* f, int mode) {
  Family& F = c->fam[fam];
  const long tot = (long)c->planes * c->Ng;
  Kern<k_plane_sums>::launch(c, PFD_PROF_OTHER, dim3(PCH, c->planes), dim3(WG), 0, c->stream, c->Ng, c->Mdiag, F.dshift, f,
                     mode == 0 ? 1 : 0, c->d_part, c->gate);
  Kern<k_plane_sub>::launch(c, PFD_PROF_OTHER, dim3(nblk(tot)), dim3(WG), 0, c->stream, c->Ng, c->planes, c->Mdiag, F.dshift,
                     c->d_part, c->Mtot, mode, f, c->gate);
}

// A convergence test that is off (plain residual or apply)
static Chk no_chk() {
  Chk k{};
  return k;
}

// r = b - A x (apply_only: r = A x) on np planes from b, x, r and the per-plane shifts sh
// (default: all planes of the family); ck: the refinement's convergence test, or none.
// Returns the number of work-groups (partial sums of the test).
static long residual(pfd_ctx* c, int fam, const double* b, const double* x, double* r, int apply_only,
                     const Chk* ck = nullptr, const double* shift = nullptr, int np = 0) {
  Family& F = c->fam[fam];
  const double* sh = shift ? shift : F.dshift;
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  const int planes = np > 0 ? np : c->planes;   // np: stacked components as extra planes
  const long tot = (long)planes * c->Ng;
  const size_t lds = sizeof(double) * (size_t)res_rows_lds(c->K, c->Nx);
  const bool tiled = c->Nx <= 256 && lds <= 64 * 1024 && (c->resid_variant == 1 || c->resid_variant == 2);
  const Chk k = ck ? *ck : no_chk();
  if (c->resid_variant == 3) {   // per node, the order a runtime argument: one kernel for every order
    Kern<k_residual<0>>::launch(c, PFD_PROF_RESID, dim3(nblk(tot)), dim3(WG), 0, c->stream, c->Nx, c->Ny, planes,
                                (int)dx.periodic, dx.dKb, dx.dM1, dx.ddir, dy.dKb, dy.dM1, dy.ddir, sh, b, x, r,
                                apply_only, c->lift[fam].ebot, k, c->K);
    return (long)nblk(tot);
  }
#define RES_CASE(KK)                                                                                      \
  case KK:                                                                                                \
    if (tiled)                                                                                            \
      Kern<k_residual_lds<KK>>::launch(c, PFD_PROF_RESID, dim3((c->Ny + RROWS - 1) / RROWS, planes), dim3(256), lds,     \
             c->stream, c->Nx, c->Ny, (int)dx.periodic, dx.dKb, dx.dM1, dx.ddir, dy.dKb, dy.dM1, dy.ddir, sh, b, x, \
             r, apply_only, c->lift[fam].ebot, k);                                                        \
    else                                                                                                  \
      Kern<k_residual<KK>>::launch(c, PFD_PROF_RESID, dim3(nblk(tot)), dim3(WG), 0, c->stream, c->Nx, c->Ny, planes,    \
             (int)dx.periodic, dx.dKb, dx.dM1, dx.ddir, dy.dKb, dy.dM1, dy.ddir, sh, b, x, r, apply_only,     \
             c->lift[fam].ebot, k, KK);                                                                   \
    break;
  switch (c->K) {
    RES_CASE(2) RES_CASE(3) RES_CASE(4) RES_CASE(5) RES_CASE(6) RES_CASE(7) RES_CASE(8) RES_CASE(9)
    RES_CASE(10) RES_CASE(11) RES_CASE(12) RES_CASE(13) RES_CASE(14) RES_CASE(15) RES_CASE(16)
  }
#undef RES_CASE
  return tiled ? (long)((c->Ny + RROWS - 1) / RROWS) * planes : (long)nblk(tot);
}

hipError_t apply(pfd_ctx* c, int fam, const double* x, double* y, int ncomp) {
  const long tot = (long)c->planes * c->Ng;
  for (int comp = 0; comp < ncomp; ++comp) residual(c, fam, nullptr, x + comp * tot, y + comp * tot, 1, nullptr);
  return hipGetLastError();
}

// the float or the double copy of an operator matrix
template <typename T>
static const T* pick(const float* f, const double* d);
template <>
const float* pick<float>(const float* f, const double*) { return f; }
template <>
const double* pick<double>(const float*, const double* d) { return d; }

// Fused middle passes of the fast-diagonalisation correction on a block of CW = 16 TN columns
// (flattened over planes, as in k_gemm_sl):
//   U = (Sy^T T1) ./ (ly_i + lx_j + c_p)   (0 where the denominator vanishes)
//   T3 = Sy U
// with the T1 block and U kept in LDS, so the intermediate never goes to memory and one launch
// replaces two.  The shared matrices come pre-arranged in MFMA fragment order (frag_layout:
// for every 16x16 tile (mt, sl) and lane, the four contraction entries the lane multiplies
// are consecutive), so a lane reads each fragment with one vector load; the next slice is
// loaded while the current one is multiplied.  Wave w takes row tiles w, w + nw, ...
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(const float* p, float (&o)[4]) {
    const V v = *reinterpret_cast<const V*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <>
struct Vec4<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load(const double* p, double (&o)[4]) {
    const V a = reinterpret_cast<const V*>(p)[0], b = reinterpret_cast<const V*>(p)[1];
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};

#define FDM_MID_LDC(CW) ((CW) + 4)

// 16-slices per prefetched chunk of fragments: 4 in FP32, 2 in FP64 (seven waves per SIMD, so
// three 9-wave work-groups share a CU)
template <typename T>
struct MidCh {
  static constexpr int v = sizeof(T) == 8 ? 2 : 4;
};

// fragments of MidCh<T>::v consecutive slices from c0 for the wave's row tiles (clamped in
// range; slices past KS and tiles past MT are not multiplied)
template <typename T, int RT>
__device__ __forceinline__ void fdm_mid_load(const T* __restrict__ Aw, int c0, int KS, int MT, int nw, int w,
                                             int lane, T (&aa)[MidCh<T>::v][RT][4]) {
#pragma unroll
  for (int q = 0; q < MidCh<T>::v; ++q) {
    const int sl = min(c0 + q, KS - 1);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int mt = min(w + nw * rt, MT - 1);
      Vec4<T>::load(Aw + ((long)(mt * KS + sl) * 64 + lane) * 4, aa[q][rt]);
    }
  }
}

// one pass acc = Aw (fragment order) x Bl (LDS); a holds the first chunk (fdm_mid_load(.., 0, ..))
template <typename T, int RT, int TN>
__device__ __forceinline__ void fdm_mid_pass(const T* __restrict__ Aw, const T* Bl, int KS, int MT, int nw, int w,
                                             int lane, T (&a)[MidCh<T>::v][RT][4],
                                             typename Mfma<T>::V (&acc)[RT][TN]) {
  typedef typename Mfma<T>::V V;
  constexpr int LDC = FDM_MID_LDC(16 * TN), CH = MidCh<T>::v;
  const int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < TN; ++ct) acc[rt][ct] = V{T(0), T(0), T(0), T(0)};
  T an[CH][RT][4];
  for (int c0 = 0; c0 < KS; c0 += CH) {
    if (c0 + CH < KS) fdm_mid_load<T, RT>(Aw, c0 + CH, KS, MT, nw, w, lane, an);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int sl = c0 + q;
      if (sl < KS) {
        T b[TN][4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int ct = 0; ct < TN; ++ct) b[ct][s] = Bl[(16 * sl + 4 * g + s) * LDC + 16 * ct + r16];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          if (w + nw * rt < MT) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int ct = 0; ct < TN; ++ct) acc[rt][ct] = Mfma<T>::op(a[q][rt][s], b[ct][s], acc[rt][ct]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s = 0; s < 4; ++s) a[q][rt][s] = an[q][rt][s];
  }
}

// One row tile per wave (RT = 1) is held to 72 VGPRs (seven waves per SIMD): at 129 rows (nine
// row tiles, so nine waves per work-group) three work-groups then fit a CU (27 of 28 wave
// slots), and the grid of a 128-plane solve runs in one round.
template <typename T, int RT, int TN>
__device__ __forceinline__ void k_fdm_mid_run(const VGrid& vg, int planes, int Ny, int Nx, long Ng,
                                              const T* __restrict__ SyTw, const T* __restrict__ Syw,
                                              const T* __restrict__ T1, const double* __restrict__ ly,
                                              const double* __restrict__ lx, const double* __restrict__ shift,
                                              T* __restrict__ T3, int ldo, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef typename Mfma<T>::V V;
  constexpr int CW = 16 * TN, LDC = FDM_MID_LDC(CW);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int KP = (Ny + 15) & ~15, MT = KP / 16;
  T* Bt = reinterpret_cast<T*>(smem_raw);   // [KP][LDC]  T1 block (rows >= Ny zero)
  T* Us = Bt + KP * LDC;                    // [KP][LDC]  U block
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6, nt = blockDim.x;
  const int r16 = lane & 15, g = lane >> 4;
  const long ctot = (long)planes * Nx, c0 = (long)vg.b.x * CW;
  T afr[MidCh<T>::v][RT][4];   // the first fragments of Sy^T are in flight while T1 is staged
  fdm_mid_load<T, RT>(SyTw, 0, MT, MT, nw, w, lane, afr);
  // stage the T1 block (coalesced along the columns), SU loads in flight per thread (column
  // indices fit an int: the launcher checks planes * Nx)
  constexpr int SU = sizeof(T) == 8 ? 4 : 8;
  const int ctoti = (int)ctot, c0i = (int)c0;
  for (int base = 0; base < KP * CW; base += SU * nt) {
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = min(base + (int)threadIdx.x + nt * u, KP * CW - 1);
      const int k = idx / CW, j = idx - k * CW;
      const int ci = c0i + j;
      const bool ok = k < Ny && ci < ctoti;
      const int cc = ci < ctoti ? ci : ctoti - 1;
      const int p = cc / Nx;
      const T x = T1[p * Ng + (long)(k < Ny ? k : Ny - 1) * Nx + (cc - p * Nx)];
      v[u] = ok ? x : T(0);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = min(base + (int)threadIdx.x + nt * u, KP * CW - 1);
      const int k = idx / CW, j = idx - k * CW;
      Bt[k * LDC + j] = v[u];
    }
  }
  __syncthreads();
  V acc[RT][TN];
  fdm_mid_pass<T, RT, TN>(SyTw, Bt, MT, MT, nw, w, lane, afr, acc);
  fdm_mid_load<T, RT>(Syw, 0, MT, MT, nw, w, lane, afr);   // in flight during the division
  // U = acc ./ (ly_i + lx_n + c_p) into LDS (rows >= Ny and columns past the end: 0)
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int mt = w + nw * rt;
    if (mt >= MT) continue;
#pragma unroll
    for (int ct = 0; ct < TN; ++ct) {
      const int j = 16 * ct + r16;
      const int ci = c0i + j;
      const int cc = ci < ctoti ? ci : ctoti - 1;
      const int p = cc / Nx;
      const int n = cc - p * Nx;
      const double lxs = lx[n] + shift[p];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * mt + Mfma<T>::row(g, q);
        const int ic = i < Ny ? i : Ny - 1;
        const double den = ly[ic] + lxs;
        const T u = (i < Ny && ci < ctoti && den != 0.0) ? T(double(acc[rt][ct][q]) / den) : T(0);
        Us[i * LDC + j] = u;
      }
    }
  }
  __syncthreads();
  fdm_mid_pass<T, RT, TN>(Syw, Us, MT, MT, nw, w, lane, afr, acc);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int mt = w + nw * rt;
    if (mt >= MT) continue;
#pragma unroll
    for (int ct = 0; ct < TN; ++ct) {
      const int ci = c0i + 16 * ct + r16;
      if (ci >= ctoti) continue;
      const int p = ci / Nx;
      const int n = ci - p * Nx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * mt + Mfma<T>::row(g, q);
        if (i < Ny) T3[((long)p * Ny + i) * (long)ldo + n] = acc[rt][ct][q];   // row stride ldo (>= Nx)
      }
    }
  }
}
template <typename T, int RT, int TN>
struct k_fdm_mid : KDef<&k_fdm_mid_run<T, RT, TN>, 1024, RT == 1 ? 7 : 1> {};

// launch of k_fdm_mid for the y-direction operator dy; false if it does not apply (LDS)
template <typename T>
static bool fdm_mid_launch(pfd_ctx* c, const Dir1D& dx, const Dir1D& dy, const double* shift, int P, const T* t1,
                           T* t3, int tn, int ldo) {
  const int Ny = c->Ny, Nx = c->Nx;
  const int KP = (Ny + 15) & ~15, MT = KP / 16;
  const int RT = (MT + 15) / 16;
  const int nw = (MT + RT - 1) / RT;
  const size_t lds = 2 * sizeof(T) * (size_t)KP * FDM_MID_LDC(16 * tn);
  if (lds > GEMM_LDS_MAX || RT > 2 || (RT == 2 && sizeof(T) == 8) || (tn != 1 && tn != 2)) return false;
  const T* SyTw = pick<T>(dy.fSTw, dy.dSTw);
  const T* Syw = pick<T>(dy.fSw, dy.dSw);
  const long ctot = (long)P * Nx;
  if (ctot + 64 > INT_MAX) return false;   // the kernel indexes columns with ints
  const dim3 grid((unsigned)((ctot + 16 * tn - 1) / (16 * tn))), block(64 * nw);
  const int cls = sizeof(T) == 8 ? PFD_PROF_GEMM64 : PFD_PROF_GEMM32;
#define MID_CASE(RT_, TN_)                                                                                   \
  if (RT == RT_ && tn == TN_)                                                                                \
    Kern<k_fdm_mid<T, RT_, TN_>>::launch(c, cls, grid, block, lds, c->stream, P, Ny, Nx, c->Ng, SyTw, Syw, t1, dy.dlam, \
           dx.dlam, shift, t3, ldo, c->gate);
  MID_CASE(1, 1) MID_CASE(1, 2)
  if constexpr (sizeof(T) == 4) {   // two row tiles per wave only where the FP32 block fits
    MID_CASE(2, 1) MID_CASE(2, 2)
  }
#undef MID_CASE
  return true;
}

// The refined path's FP64 residual of RROWS rows fused with the first fast-diagonalisation
// pass: T1[rows] = float(b - A x)[rows] Sx.  The residual rows (res_rows) go to LDS in FP32,
// zero past Ny and Nx, and the rows x Sx product runs on the matrix cores, each wave taking
// column tiles w, w + 4, ...  Sx comes in B-fragment order, which is the fragment order of
// Sx^T as a left operand (frag_layout of S^T): for column tile nt, slice sl and lane, the four
// entries Sx[16 sl + 4 (lane / 16) + s][16 nt + lane % 16].
// NTW: column tiles per wave, ceil(KPX / 64) (3 up to Nx = 192, 4 up to 256).
template <int K, int NTW>
__device__ __forceinline__ void k_res_p1_run(const VGrid& vg, int Nx, int Ny, int perx,
                                             const double* __restrict__ KxB, const double* __restrict__ Mx,
                                             const unsigned char* __restrict__ dirx, const double* __restrict__ KyB,
                                             const double* __restrict__ My, const unsigned char* __restrict__ diry,
                                             const double* __restrict__ shift, const double* __restrict__ bb,
                                             const double* __restrict__ x, const unsigned char* __restrict__ ebot,
                                             const float* __restrict__ SxB, float* __restrict__ T1, Chk ck) {
  if (ck.gin && *ck.gin) return;
  typedef Mfma<float>::V V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xs = reinterpret_cast<double*>(smem_raw);
  const int KPX = (Nx + 15) & ~15, KS = KPX / 16, LDR = KPX + 4;
  float* Rl = reinterpret_cast<float*>(xs + res_rows_lds(K, Nx));   // [RROWS][LDR]
  for (int idx = threadIdx.x; idx < RROWS * LDR; idx += 256) Rl[idx] = 0.0f;
  __syncthreads();   // zero fill before the residual rows land (res_rows syncs after its staging)
  double r2 = 0.0, x2 = 0.0;
  res_rows<K>(vg, Nx, Ny, perx, KxB, Mx, dirx, KyB, My, diry, shift, bb, x, 0, ebot, xs,
              [&](int rl, int, int ix, double v, double bv, double xv) {
                Rl[rl * LDR + ix] = float(v);
                r2 += v * v;
                x2 += xv * xv;
              });
  if (ck.part) {   // the test's sums leave the registers before the matrix-core phase
    int rb0, pl0;
    xcd_tile(vg, rb0, pl0);
    const double an = ck.anorm[pl0 % ck.nplane];
    chk_store(vg, ck, r2, an * an * x2);
  }
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int NT = KS;   // column tiles of the square product
  V acc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) acc[j] = V{0.f, 0.f, 0.f, 0.f};
  constexpr int CH = 4;   // slices per prefetched chunk of Sx fragments
  float bq[CH][NTW][4], bn[CH][NTW][4];
  auto loadB = [&](int c0, float (&bb)[CH][NTW][4]) {   // clamped; past KS / NT not multiplied
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int sl = min(c0 + q, KS - 1);
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        const int nt = min(w + 4 * j, NT - 1);
        Vec4<float>::load(SxB + ((long)(nt * KS + sl) * 64 + lane) * 4, bb[q][j]);
      }
    }
  };
  loadB(0, bq);   // the first Sx fragments are in flight while the other waves finish their rows
  __syncthreads();
  for (int c0 = 0; c0 < KS; c0 += CH) {
    if (c0 + CH < KS) loadB(c0 + CH, bn);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int sl = c0 + q;
      if (sl < KS) {
        const Mfma<float>::V av = *reinterpret_cast<const Mfma<float>::V*>(Rl + r16 * LDR + 16 * sl + 4 * g);
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
          if (w + 4 * j < NT) {
            acc[j] = Mfma<float>::op(av.x, bq[q][j][0], acc[j]);
            acc[j] = Mfma<float>::op(av.y, bq[q][j][1], acc[j]);
            acc[j] = Mfma<float>::op(av.z, bq[q][j][2], acc[j]);
            acc[j] = Mfma<float>::op(av.w, bq[q][j][3], acc[j]);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
#pragma unroll
      for (int j = 0; j < NTW; ++j)
#pragma unroll
        for (int k = 0; k < 4; ++k) bq[q][j][k] = bn[q][j][k];
  }
  int rb, pl;
  xcd_tile(vg, rb, pl);   // the tile res_rows took
  const long Ng = (long)Nx * Ny, pofs = (long)pl * Ng;
  const int iy0 = rb * RROWS;
#pragma unroll
  for (int j = 0; j < NTW; ++j) {
    const int nt = w + 4 * j;
    const int n = 16 * nt + r16;
    if (nt >= NT || n >= Nx) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int iy = iy0 + Mfma<float>::row(g, q);
      if (iy < Ny) T1[pofs + (long)iy * Nx + n] = acc[j][q];
    }
  }
}
template <int K, int NTW>
struct k_res_p1 : KDef<&k_res_p1_run<K, NTW>, 256, K <= 8 && NTW == 3 ? 3 : 1> {};

// Last fast-diagonalisation pass of the refined path, x (+)= T3 Sx^T, after k_fdm_mid wrote T3
// (FP32) with the padded row stride KPX = Nx rounded up to 16: a lane then reads each A fragment
// (four consecutive contraction entries of its row) with one 16-byte load, and Sx^T comes as
// right operand in fragment order (which is the fragment order of Sx as a left operand).  A wave
// takes one 16-row tile of the flattened planes x rows and TG column tiles; contraction entries
// past Nx are masked to zero; fragments come CH slices per prefetched chunk.  EPI 2: x += ;
// EPI 3: x = .
template <int EPI, int TG, int CH>
__device__ __forceinline__ void k_p4_run(const VGrid& vg, const float* __restrict__ T3, int Mtot, int Nx, int KPX,
                                         const float* __restrict__ SxFw, double* __restrict__ X,
                                         const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef Mfma<float>::V V;
  const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
  const int KS = KPX / 16, NT = KS, NG = (NT + TG - 1) / TG, MT = (Mtot + 15) / 16;
  const int wid = __builtin_amdgcn_readfirstlane((int)(vg.b.x * 4 + (threadIdx.x >> 6)));
  const int rt = wid / NG, grp = wid - rt * NG;
  if (rt >= MT) return;   // no barrier in this kernel: a whole wave leaves
  const int m = min(16 * rt + r16, Mtot - 1);   // clamped row; rows past Mtot are not stored
  const float* Ar = T3 + (long)m * KPX + 4 * g;
  V acc[TG];
#pragma unroll
  for (int j = 0; j < TG; ++j) acc[j] = V{0.f, 0.f, 0.f, 0.f};
  float a[CH][4], an[CH][4], b[CH][TG][4], bn[CH][TG][4];
  auto load = [&](int c0, float (&aa)[CH][4], float (&bb)[CH][TG][4]) {
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int sl = min(c0 + q, KS - 1);
      Vec4<float>::load(Ar + 16 * sl, aa[q]);
#pragma unroll
      for (int j = 0; j < TG; ++j) {
        const int nt = min(grp * TG + j, NT - 1);
        Vec4<float>::load(SxFw + ((long)(nt * KS + sl) * 64 + lane) * 4, bb[q][j]);
      }
    }
  };
  load(0, a, b);
  for (int c0 = 0; c0 < KS; c0 += CH) {
    if (c0 + CH < KS) load(c0 + CH, an, bn);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int sl = c0 + q;
      if (sl < KS) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float av = (16 * sl + 4 * g + s < Nx) ? a[q][s] : 0.f;   // padding columns
#pragma unroll
          for (int j = 0; j < TG; ++j)
            if (grp * TG + j < NT) acc[j] = Mfma<float>::op(av, b[q][j][s], acc[j]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
#pragma unroll
      for (int s = 0; s < 4; ++s) a[q][s] = an[q][s];
#pragma unroll
      for (int j = 0; j < TG; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) b[q][j][s] = bn[q][j][s];
    }
  }
#pragma unroll
  for (int j = 0; j < TG; ++j) {
    const int nt = grp * TG + j;
    const int n = 16 * nt + r16;
    if (nt >= NT || n >= Nx) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int mm = 16 * rt + Mfma<float>::row(g, q);
      if (mm >= Mtot) continue;
      if (EPI == 2) X[(long)mm * Nx + n] += double(acc[j][q]);
      else X[(long)mm * Nx + n] = double(acc[j][q]);
    }
  }
}
template <int EPI, int TG, int CH>
struct k_p4 : KDef<&k_p4_run<EPI, TG, CH>, 256, 0> {};

// k_p4 over P planes (tg column tiles per wave); false where it does not apply
// form: 1..4 column tiles per wave with two-slice chunks, 6 one tile with four-slice chunks
static bool p4_launch(pfd_ctx* c, const Dir1D& dx, int P, const float* t3, double* x, bool overwrite, int form) {
  const int Nx = c->Nx, KPX = (Nx + 15) & ~15, NT = KPX / 16;
  if (!((form >= 1 && form <= 4) || form == 6)) return false;
  const int tg = form == 6 ? 1 : form;
  const long Mtot = (long)P * c->Ny;
  const long waves = ((Mtot + 15) / 16) * ((NT + tg - 1) / tg);
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define P4_CASE(F_, TG_, CH_)                                                                                 \
  if (form == F_) {                                                                                           \
    if (overwrite)                                                                                            \
      Kern<k_p4<3, TG_, CH_>>::launch(c, PFD_PROF_GEMM32, grid, block, 0, c->stream, t3, (int)Mtot, Nx, KPX, dx.fSw, x, \
             c->gate);                                                                                        \
    else                                                                                                      \
      Kern<k_p4<2, TG_, CH_>>::launch(c, PFD_PROF_GEMM32, grid, block, 0, c->stream, t3, (int)Mtot, Nx, KPX, dx.fSw, x, \
             c->gate);                                                                                        \
  }
  P4_CASE(1, 1, 2) P4_CASE(2, 2, 2) P4_CASE(3, 3, 2) P4_CASE(4, 4, 2) P4_CASE(6, 1, 4)
#undef P4_CASE
  return true;
}

// First / last fast-diagonalisation pass of the refined path with the shared matrix resident in
// LDS for the whole launch: C = A S, A (Mtot x K, row stride lda, FP64 or FP32) times S (K x N,
// B-fragment order, i.e. the fragment order of S^T as a left operand), one work-group per CU
// looping over 16-row tiles of A (staged through LDS in FP32, coalesced; the next tile is
// loaded while the current one is multiplied), wave w taking column tiles w, w + nw, ...  The
// matrix (up to 320^2 FP32) is read from L2 once per work-group instead of once per tile.
// EPI 0: C = acc (FP32, row stride ldc); 2: X += acc; 3: X = acc.  Needs K, N <= 32 * 16.
template <typename TA, int EPI>
__device__ __forceinline__ void k_srp_run(const VGrid& vg, const TA* __restrict__ A, int lda, int Mtot, int K, int N,
                                          const float* __restrict__ SB, float* __restrict__ C, double* __restrict__ X,
                                          int ldc, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  typedef Mfma<float>::V V;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int KP = (K + 15) & ~15, KS = KP / 16, NT = (N + 15) / 16, LDA = KP + 4;
  float* Sl = reinterpret_cast<float*>(smem_raw);   // NT * KS * 256 (fragment order)
  float* Al = Sl + (long)NT * KS * 256;             // [16][LDA]
  const int nt_thr = blockDim.x, tid = threadIdx.x;
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nt_thr >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  for (int idx = 4 * tid; idx < NT * KS * 256; idx += 4 * nt_thr)
    *reinterpret_cast<V*>(Sl + idx) = *reinterpret_cast<const V*>(SB + idx);
  const int MT = (Mtot + 15) / 16;
  // a tile's 16 x KP values take one round of at most 8 per thread (16 KP <= 8 * 64 nw); the
  // next tile's are loaded into registers while the current one is multiplied
  float v[8];
  auto load_tile = [&](int t) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = min(tid + nt_thr * u, 16 * KP - 1);
      const int r = idx / KP, k = idx - r * KP;
      const int m = 16 * t + r;
      const bool ok = m < Mtot && k < K;
      const float x = float(A[(long)(m < Mtot ? m : Mtot - 1) * lda + (k < K ? k : K - 1)]);
      v[u] = ok ? x : 0.f;
    }
  };
  if (vg.b.x < MT) load_tile(vg.b.x);
  for (int t = vg.b.x; t < MT; t += vg.g.x) {
    __syncthreads();   // the matrix is staged / the previous tile's rows are read
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + nt_thr * u;
      if (idx < 16 * KP) {
        const int r = idx / KP, k = idx - r * KP;
        Al[r * LDA + k] = v[u];
      }
    }
    __syncthreads();
    if (t + (int)vg.g.x < MT) load_tile(t + vg.g.x);
    for (int nt = w; nt < NT; nt += nw) {
      // two accumulators (even and odd slices) halve the dependent chain of matrix-core ops
      V acc = V{0.f, 0.f, 0.f, 0.f}, acc1 = V{0.f, 0.f, 0.f, 0.f};
      int sl = 0;
      for (; sl + 1 < KS; sl += 2) {
        const V a4 = *reinterpret_cast<const V*>(Al + r16 * LDA + 16 * sl + 4 * g);
        const V b4 = *reinterpret_cast<const V*>(Sl + ((long)(nt * KS + sl) * 64 + lane) * 4);
        const V a5 = *reinterpret_cast<const V*>(Al + r16 * LDA + 16 * sl + 16 + 4 * g);
        const V b5 = *reinterpret_cast<const V*>(Sl + ((long)(nt * KS + sl + 1) * 64 + lane) * 4);
        acc = Mfma<float>::op(a4.x, b4.x, acc);
        acc1 = Mfma<float>::op(a5.x, b5.x, acc1);
        acc = Mfma<float>::op(a4.y, b4.y, acc);
        acc1 = Mfma<float>::op(a5.y, b5.y, acc1);
        acc = Mfma<float>::op(a4.z, b4.z, acc);
        acc1 = Mfma<float>::op(a5.z, b5.z, acc1);
        acc = Mfma<float>::op(a4.w, b4.w, acc);
        acc1 = Mfma<float>::op(a5.w, b5.w, acc1);
      }
      if (sl < KS) {
        const V a4 = *reinterpret_cast<const V*>(Al + r16 * LDA + 16 * sl + 4 * g);
        const V b4 = *reinterpret_cast<const V*>(Sl + ((long)(nt * KS + sl) * 64 + lane) * 4);
        acc = Mfma<float>::op(a4.x, b4.x, acc);
        acc = Mfma<float>::op(a4.y, b4.y, acc);
        acc = Mfma<float>::op(a4.z, b4.z, acc);
        acc = Mfma<float>::op(a4.w, b4.w, acc);
      }
      acc += acc1;
      const int n = 16 * nt + r16;
      if (n >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = 16 * t + Mfma<float>::row(g, q);
        if (m >= Mtot) continue;
        if (EPI == 0) C[(long)m * ldc + n] = acc[q];
        else if (EPI == 2) X[(long)m * ldc + n] += double(acc[q]);
        else X[(long)m * ldc + n] = double(acc[q]);
      }
    }
  }
}
template <typename TA, int EPI>
struct k_srp : KDef<&k_srp_run<TA, EPI>, 1024, 0> {};

// bytes of LDS k_srp needs for a K x N matrix; 0 where it exceeds what a work-group may have
static size_t srp_lds(pfd_ctx* c, int K, int N) {
  const size_t KP = (K + 15) & ~15, NT = (N + 15) / 16;
  const size_t b = sizeof(float) * (NT * 16 * KP + 16 * (KP + 4));
  if (16 * KP > 8 * 64 * std::min<size_t>(NT, 16)) return 0;   // one register round per tile
  return b <= (size_t)c->lds_max ? b : 0;
}

// k_srp over P planes of Ny rows; false where it does not apply
template <typename TA, int EPI>
static bool srp_launch(pfd_ctx* c, int P, const TA* A, int lda, int K, int N, const float* SB, float* C, double* X,
                       int ldc) {
  const size_t lds = srp_lds(c, K, N);
  if (!lds) return false;
  const int Mtot = P * c->Ny, MT = (Mtot + 15) / 16, NT = (N + 15) / 16;
  const int nw = NT < 16 ? NT : 16;
  const unsigned grid = (unsigned)std::min(MT, c->num_cu);
  Kern<k_srp<TA, EPI>>::launch(c, PFD_PROF_GEMM32, dim3(grid), dim3(64 * nw), lds, c->stream, A, lda, Mtot, K, N, SB, C, X,
         ldc, c->gate);
  return true;
}

// refined path: T1 = float(b - A x) Sx for family fam in one launch (k_res_p1); false where it
// does not apply (Nx > 256 or the LDS tile too large)
static bool res_p1_launch(pfd_ctx* c, int fam, const double* b, const double* x, const double* shift, int np,
                          float* t1, const Chk& ck) {
  Family& F = c->fam[fam];
  const Dir1D& dx = c->dirs[F.ix];
  const Dir1D& dy = c->dirs[F.iy];
  const int KPX = (c->Nx + 15) & ~15;
  const size_t lds = sizeof(double) * (size_t)res_rows_lds(c->K, c->Nx) + sizeof(float) * RROWS * (KPX + 4);
  if (c->Nx > 256 || lds > 64 * 1024) return false;
  const dim3 grid((c->Ny + RROWS - 1) / RROWS, np);
  const bool three = KPX <= 192;   // column tiles per wave
#define RP1_CASE(KK)                                                                                         \
  case KK:                                                                                                   \
    if (three)                                                                                               \
      Kern<k_res_p1<KK, 3>>::launch(c, PFD_PROF_RESID, grid, dim3(256), lds, c->stream, c->Nx, c->Ny, (int)dx.periodic, \
             dx.dKb, dx.dM1, dx.ddir, dy.dKb, dy.dM1, dy.ddir, shift, b, x, c->lift[fam].ebot,                 \
             (const float*)dx.fSTw, t1, ck);                                                                 \
    else                                                                                                     \
      Kern<k_res_p1<KK, 4>>::launch(c, PFD_PROF_RESID, grid, dim3(256), lds, c->stream, c->Nx, c->Ny, (int)dx.periodic, \
             dx.dKb, dx.dM1, dx.ddir, dy.dKb, dy.dM1, dy.ddir, shift, b, x, c->lift[fam].ebot,                 \
             (const float*)dx.fSTw, t1, ck);                                                                 \
    return true;
  switch (c->K) {
    RP1_CASE(2) RP1_CASE(3) RP1_CASE(4) RP1_CASE(5) RP1_CASE(6) RP1_CASE(7) RP1_CASE(8) RP1_CASE(9)
    RP1_CASE(10) RP1_CASE(11) RP1_CASE(12) RP1_CASE(13) RP1_CASE(14) RP1_CASE(15) RP1_CASE(16)
  }
#undef RP1_CASE
  return false;
}

// Fast-diagonalisation correction  x += Sy [ (Sy^T r Sx) ./ (ly_i + lx_j + c_p) ] Sx^T
// as four batched GEMMs over all planes (Sx, Sy shared by every plane); variant 1: two fused
// strip kernels; variant 2: the two middle passes fused (three launches).
template <typename T>
static void fdm_correct(pfd_ctx* c, const Dir1D& dx, const Dir1D& dy, const double* shift, const T* Sx,
                        const T* SxT, const T* Sy, const T* SyT, const double* r, double* x,
                        bool overwrite = false, int np = 0, bool t1_ready = false) {
  const int Nx = c->Nx, Ny = c->Ny, P = np > 0 ? np : c->planes;   // np: stacked components
  const long Ng = c->Ng;
  T* t1 = reinterpret_cast<T*>(c->tmp);
  T* t2 = reinterpret_cast<T*>(c->tmp2);
  if (c->fdm_variant == 1) {
    const int cls = sizeof(T) == 8 ? PFD_PROF_GEMM64 : PFD_PROF_GEMM32;
    Kern<k_fdm1<T>>::launch(c, cls, dim3(P * ((Nx + 15) / 16)), dim3(256), 0, c->stream, P, Ny, Nx, Ng, r, SxT, SyT,
           dy.dlam, dx.dlam, shift, t1, c->gate);
    if (overwrite)
      Kern<k_fdm2<T, true>>::launch(c, cls, dim3(P * ((Ny + 15) / 16)), dim3(256), 0, c->stream, P, Ny, Nx, Ng,
             (const T*)t1, Sy, Sx, x, c->gate);
    else
      Kern<k_fdm2<T, false>>::launch(c, cls, dim3(P * ((Ny + 15) / 16)), dim3(256), 0, c->stream, P, Ny, Nx, Ng,
             (const T*)t1, Sy, Sx, x, c->gate);
    return;
  }
  if (!t1_ready) {   // else the first pass came with the residual (k_res_p1)
    bool done = false;
    if constexpr (sizeof(T) == 4)
      done = c->p1_srp && srp_launch<double, 0>(c, P, r, Nx, Nx, Nx, dx.fSTw, t1, nullptr, Nx);
    if (!done)
      gemm<T, double, T, 0>(c, PFD_GS_P1, P, r, Ng, Sx, 0, Ny, Nx, Nx, t1, Ng, nullptr, nullptr, nullptr, nullptr);
  }
  // refined path with the fused middle passes: T3 with the padded row stride for k_p4
  // (the padded FP32 block must fit the scratch buffer: 3 planes-worth of FP64 fields)
  const bool pad = sizeof(T) == 4 && c->fdm_variant == 2 && c->p4_tg > 0 &&
                   (long)P * Ny * ((Nx + 15) & ~15) <= 6L * c->planes * Ng;
  if (!(c->fdm_variant == 2 && fdm_mid_launch<T>(c, dx, dy, shift, P, t1, t2, c->mid_tn,
                                                 pad ? ((Nx + 15) & ~15) : Nx))) {
    gemm<T, T, T, 1>(c, PFD_GS_P2, P, SyT, 0, t1, Ng, Ny, Nx, Ny, t2, Ng, dy.dlam, dx.dlam, shift, nullptr);
    gemm<T, T, T, 0>(c, PFD_GS_P3, P, Sy, 0, t2, Ng, Ny, Nx, Ny, t1, Ng, nullptr, nullptr, nullptr, nullptr);
  } else {
    if (pad) {
      if constexpr (sizeof(T) == 4) {
        const int KPX = (Nx + 15) & ~15;
        if (c->p4_tg == 5 && (overwrite ? srp_launch<float, 3>(c, P, t2, KPX, Nx, Nx, dx.fSw, nullptr, x, Nx)
                                        : srp_launch<float, 2>(c, P, t2, KPX, Nx, Nx, dx.fSw, nullptr, x, Nx)))
          return;
        p4_launch(c, dx, P, t2, x, overwrite, c->p4_tg == 5 ? 1 : c->p4_tg);   // reads the padded rows
        return;
      }
    }
    std::swap(t1, t2);   // the fused passes wrote T3 to t2
  }
  if constexpr (sizeof(T) == 4) {
    if (c->p4_tg == 5 && (overwrite ? srp_launch<float, 3>(c, P, t1, Nx, Nx, Nx, dx.fSw, nullptr, x, Nx)
                                    : srp_launch<float, 2>(c, P, t1, Nx, Nx, Nx, dx.fSw, nullptr, x, Nx)))
      return;
  }
  if (overwrite)
    gemm<T, T, T, 3>(c, PFD_GS_P4, P, t1, Ng, SxT, 0, Ny, Nx, Nx, (T*)nullptr, Ng, nullptr, nullptr, nullptr, x);
  else
    gemm<T, T, T, 2>(c, PFD_GS_P4, P, t1, Ng, SxT, 0, Ny, Nx, Nx, (T*)nullptr, Ng, nullptr, nullptr, nullptr, x);
}

// Electrode gap nodes (potential family): with Y = A_FF^{-1} r_F from the base operator,
//   t_G = r_G - A_GF Y,  dG = S_G^{-1} t_G  (S_G^{-1} per plane, FP64, from set-up)
// where A_GF Y at gap node (g, 0) = Mx[g] sum_{iy=1..K} Ky[0][iy] Y(g, iy).
__device__ __forceinline__ void k_elec_gap_run(const VGrid& vg, int Nx, int Ny, int K, long Ng, int ng,
                                               const int* __restrict__ gap, const double* __restrict__ Mx,
                                               const double* __restrict__ Ky0, const double* __restrict__ r,
                                               const double* __restrict__ Y, const double* __restrict__ Sinv,
                                               double* __restrict__ dG, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  __shared__ double t[PFD_NMAX];
  const int pl = vg.b.x;
  const double* rp = r + pl * Ng;
  const double* Yp = Y + pl * Ng;
  const int kmax = min(K, Ny - 1);
  for (int i = threadIdx.x; i < ng; i += blockDim.x) {
    const int gx = gap[i];
    double acc = 0.0;
    for (int iy = 1; iy <= kmax; ++iy) acc += Ky0[iy] * Yp[(long)iy * Nx + gx];
    t[i] = rp[gx] - Mx[gx] * acc;
  }
  __syncthreads();
  const double* Sp = Sinv + (long)pl * ng * ng;
  for (int i = threadIdx.x; i < ng; i += blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < ng; ++j) acc += Sp[(long)i * ng + j] * t[j];
    dG[(long)pl * ng + i] = acc;
  }
}
struct k_elec_gap : KDef<&k_elec_gap_run, 0, 0> {};

// z = -A_FG dG (nonzero in the gap columns, rows 1..K), and x += Y (+ dG on the gap nodes)
__device__ __forceinline__ void k_elec_z_run(const VGrid& vg, int Nx, int Ny, int K, int planes, int ng,
                                             const int* __restrict__ gapidx, const double* __restrict__ Mx,
                                             const double* __restrict__ Ky0, const double* __restrict__ dG,
                                             const double* __restrict__ Y, double* __restrict__ z,
                                             double* __restrict__ x, const int* __restrict__ gate) {
  if (gate && *gate) return;   // the refinement has converged: nothing left to do
  const long Ng = (long)Nx * Ny;
  const long id = (long)vg.b.x * blockDim.x + threadIdx.x;
  if (id >= planes * Ng) return;
  const int pl = (int)(id / Ng);
  const int node = (int)(id - pl * Ng);
  const int iy = node / Nx, ix = node - iy * Nx;
  const int i = gapidx[ix];
  double zv = 0.0, add = Y[id];
  if (i >= 0) {
    const double d = dG[(long)pl * ng + i];
    if (iy >= 1 && iy <= K) zv = -Mx[ix] * Ky0[iy] * d;
    if (iy == 0) add += d;
  }
  z[id] = zv;
  x[id] += add;
}
struct k_elec_z : KDef<&k_elec_z_run, 0, 0> {};

// one correction of the potential family with electrode gap nodes:
//   x += A_FF^{-1}(r_F - A_FG dG) on F,  x += dG on G
template <typename T>
static void elec_correct(pfd_ctx* c, const Dir1D& dx, const Dir1D& dy, const double* shift, const T* Sx,
                         const T* SxT, const T* Sy, const T* SyT, const double* r, double* x) {
  const long tot = (long)c->planes * c->Ng;
  double* z = c->r + tot;   // scratch block of r (the potential solve uses block 0)
  fdm_correct<T>(c, dx, dy, shift, Sx, SxT, Sy, SyT, r, c->Ybuf, true);
  Kern<k_elec_gap>::launch(c, PFD_PROF_OTHER, dim3(c->planes), dim3(WG), 0, c->stream, c->Nx, c->Ny, c->K, c->Ng,
         c->elec.ng, c->elec.d_gap, dx.dM1, dy.dK0, r, c->Ybuf, c->elec.d_Sinv, c->elec.d_dG, c->gate);
  Kern<k_elec_z>::launch(c, PFD_PROF_OTHER, dim3(nblk(tot)), dim3(WG), 0, c->stream, c->Nx, c->Ny, c->K, c->planes,
         c->elec.ng, c->elec.d_gapidx, dx.dM1, dy.dK0, c->elec.d_dG, c->Ybuf, z, x, c->gate);
  fdm_correct<T>(c, dx, dy, shift, Sx, SxT, Sy, SyT, z, x);
}

// One FP64 fast-diagonalisation correction (a direct solve) of planes [p0, p0 + np) of one
// component: x += A^{-1} r with r = b - A x formed here unless r0 (exact) is given.  project:
// the right side may be incompatible on singular planes and the guess arbitrary (general entry
// point), so the residual is projected onto the range; singular planes get the gauge
// int_h x = 0 afterwards.
static void solve64(pfd_ctx* c, int fam, const double* b, double* x, int p0, int np, int project,
                    const double* r0) {
  Family& F = c->fam[fam];
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  const bool elec = fam == PFD_FAM_V && c->elec.ng > 0;   // all planes (no plane split)
  const long o = (long)p0 * c->Ng;
  const double* sh = F.dshift + p0;
  const double* rin = r0;
  if (!rin) {
    residual(c, fam, b + o, x + o, c->r + o, 0, nullptr, sh, np);
    if (F.any_singular && project) plane_fix(c, fam, c->r, 1);
    rin = c->r + o;
  }
  if (elec)
    elec_correct<double>(c, dx, dy, F.dshift, dx.dS, dx.dST, dy.dS, dy.dST, rin, x);
  else
    fdm_correct<double>(c, dx, dy, sh, dx.dS, dx.dST, dy.dS, dy.dST, rin, x + o, false, np);
}

// FP32 corrections with FP64 residuals (iterative refinement) on planes [p0, p0 + np/ncomp) of
// ncomp stacked components (np planes in all).  r0: the first residual, recycled from the right
// sides (the first correction then takes it untested).  Every later residual is tested (Chk) and
// sets the gate; the corrections after it, and the remaining tests, return at once once it is
// set, so the whole sequence can be captured in a graph.  After refine_max corrections a last
// test records non-convergence (status bit, returned as PFD_ENOCONV by the stepping calls).
static void refine32(pfd_ctx* c, int fam, const double* b, double* x, int p0, int np, const double* r0) {
  Family& F = c->fam[fam];
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  const bool elec = fam == PFD_FAM_V && c->elec.ng > 0;
  const long o = (long)p0 * c->Ng;
  const double* sh = F.dshift + p0;
  const int per = c->planes - p0;   // planes per component in this range
  Chk ck{};
  ck.part = c->d_rpart;
  ck.anorm = c->d_anorm[fam] + p0;
  ck.nplane = per;
  // the test of the residual just formed: its partial sums -> gate and record
  auto decide = [&](long nb, int it, int last, const int* gin) {
    Kern<k_chk_decide>::launch(c, PFD_PROF_OTHER, dim3(1), dim3(256), 0, c->stream, (const double*)c->d_rpart, nb, gin,
           c->d_gate, c->d_rstat + 4 * fam, c->d_status, c->refine_tol, it, last, fam);
  };
  const int maxit = c->refine_max;
  bool tested = false;   // a test of this solve has written the gate
  for (int it = 0; it < maxit; ++it) {
    const double* rin = c->r + o;
    bool t1_ready = false;
    if (it == 0 && r0) {
      rin = r0 + o;
    } else {
      const int* gin = tested ? c->d_gate : nullptr;
      ck.gin = gin;
      long nb = (long)((c->Ny + RROWS - 1) / RROWS) * np;
      if (!elec && c->resid_variant == 2 && c->fdm_variant != 1 &&
          res_p1_launch(c, fam, b + o, x + o, sh, np, reinterpret_cast<float*>(c->tmp), ck))
        t1_ready = true;
      else
        nb = residual(c, fam, b + o, x + o, c->r + o, 0, &ck, sh, np);
      decide(nb, it, 0, gin);
      tested = true;
    }
    c->gate = tested ? c->d_gate : nullptr;
    if (elec)
      elec_correct<float>(c, dx, dy, F.dshift, dx.fS, dx.fST, dy.fS, dy.fST, rin, x);
    else
      fdm_correct<float>(c, dx, dy, sh, dx.fS, dx.fST, dy.fS, dy.fST, rin, x + o, false, np, t1_ready);
    c->gate = nullptr;
  }
  const int* gin = tested ? c->d_gate : nullptr;
  ck.gin = gin;
  const long nb = residual(c, fam, b + o, x + o, c->r + o, 0, &ck, sh, np);
  decide(nb, maxit, 1, gin);
}

// Solve (K + c M) x = b for ncomp stacked right sides (each planes*Ng), x holding the initial
// guess and the Dirichlet values.  r0 != nullptr: the first residual b - A x is given (stacked
// like b): exact on the plain FP64 path and on families the FP32-refined path solves in FP64
// (r0_exact), recycled from the right sides otherwise.  project != 0: the right side may be
// incompatible on singular planes and the initial guess arbitrary (general entry point).
// The precision ladder splits a family's planes: [0, n64) by one FP64 correction (singular
// and ill-conditioned operators), the rest by FP32 iterative refinement (refined path only).
hipError_t solve(pfd_ctx* c, int fam, const double* b, double* x, int ncomp, int project, const double* r0,
                 bool r0_exact) {
  Family& F = c->fam[fam];
  const long tot = (long)c->planes * c->Ng;
  const bool refined = c->prob.precision == PFD_REFINED_FP32;
  const int n64 = refined ? c->n64[fam] : c->planes;
  const bool elec = fam == PFD_FAM_V && c->elec.ng > 0;
  for (int comp = 0; comp < ncomp; ++comp) {
    if (n64 == 0) break;
    const double* rc = (r0 && (r0_exact || !refined)) ? r0 + comp * tot : nullptr;
    solve64(c, fam, b + comp * tot, x + comp * tot, 0, n64, project, rc);
    if (F.any_singular) plane_fix(c, fam, x + comp * tot, 0);
  }
  if (n64 < c->planes) {
    // up to three contiguous components (the velocity) are refined as one stack of planes;
    // electrode solves go one by one
    const bool stack = ncomp > 1 && ncomp <= 3 && n64 == 0 && !elec;
    const int groups = stack ? 1 : ncomp;
    const int np = (c->planes - n64) * (stack ? ncomp : 1);
    for (int gi = 0; gi < groups; ++gi)
      refine32(c, fam, b + gi * tot, x + gi * tot, n64, np, r0 ? r0 + gi * tot : nullptr);
  }
  return hipGetLastError();
}

// Back-to-back replay of one kernel class on the context's real shapes and buffers,
// bracketed by two events on its stream: average device time per launch (us).
// GEMM classes replay the four passes of one velocity-family correction into scratch;
// the residual class replays the velocity-family residual.
hipError_t replay(pfd_ctx* c, int cls, int reps, double* avg_us) {
  Family& F = c->fam[PFD_FAM_U];
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e) return e;
  e = hipEventCreate(&e1);
  if (e) return e;
  const int saved = c->prof_on;
  c->prof_on = 0;
  double* scratch = c->b[2];
  int per = 1;
  (void)hipEventRecord(e0, c->stream);
  for (int i = 0; i < reps; ++i) {
    if (cls == PFD_PROF_GEMM32) {
      fdm_correct<float>(c, dx, dy, F.dshift, dx.fS, dx.fST, dy.fS, dy.fST, c->r, scratch);
      per = c->fdm_variant == 1 ? 2 : (c->fdm_variant == 2 ? 3 : 4);
    } else if (cls == PFD_PROF_GEMM64) {
      fdm_correct<double>(c, dx, dy, F.dshift, dx.dS, dx.dST, dy.dS, dy.dST, c->r, scratch);
      per = c->fdm_variant == 1 ? 2 : (c->fdm_variant == 2 ? 3 : 4);
    } else {
      residual(c, PFD_FAM_U, c->b[1], scratch, c->r + 2 * (long)c->planes * c->Ng, 0, nullptr);
    }
  }
  (void)hipEventRecord(e1, c->stream);
  e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (!e) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->prof_on = saved;
  *avg_us = 1e3 * ms / (double(reps) * per);
  return e;
}

static void ztrans(pfd_ctx* c, const double* W, const double* in, double* out, const double* in2, double c1,
                   double c2);

// Autotuner.  For every GEMM call site (the four fast-diagonalisation passes in the context's
// solve precision, and the z transform in 3D) each tile configuration is timed on the real
// shapes with scratch operands, and the fastest is kept; then one velocity-family correction
// with the tuned passes is timed against the fused strip kernels and the faster variant kept.
// Scratch buffers only; the state is not touched.

// Holds the stream for `ticks` of the device's constant-rate wall clock (one lane; the loop ends
// when the clock has advanced that far).
__global__ void k_hold(long long ticks) {
  const long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) {
  }
}

// average time of f over reps back-to-back calls, the least of three such runs (a single run
// picked between candidates within a few per cent of each other by clock and queue noise).
// Each run starts behind a 0.5 ms hold of the stream, so the host has queued every call before
// the first one starts: small kernels are then timed back to back on the GPU, as a captured
// step replays them, not at the rate the host can launch them.
static double time_us(pfd_ctx* c, hipEvent_t e0, hipEvent_t e1, int reps, const std::function<void()>& f,
                      hipError_t& e) {
  f();
  double best = 0.0;
  for (int run = 0; run < 3 && !e; ++run) {
    hipLaunchKernelGGL(k_hold, dim3(1), dim3(1), 0, c->stream, c->hold_ticks);
    (void)hipEventRecord(e0, c->stream);
    for (int i = 0; i < reps; ++i) f();
    (void)hipEventRecord(e1, c->stream);
    e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (!e) e = hipEventElapsedTime(&ms, e0, e1);
    const double us = 1e3 * ms / reps;
    if (run == 0 || us < best) best = us;
  }
  return best;
}

template <typename T>
static void tune_fdm_sites(pfd_ctx* c, hipEvent_t e0, hipEvent_t e1, hipError_t& e) {
  Family& F = c->fam[PFD_FAM_U];
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  const int P = c->planes, Nx = c->Nx, Ny = c->Ny;
  const long Ng = c->Ng;
  const int ti = sizeof(T) == 8 ? 1 : 0;
  const int cls = ti ? PFD_PROF_GEMM64 : PFD_PROF_GEMM32;
  T* t1 = reinterpret_cast<T*>(c->tmp);
  T* t2 = reinterpret_cast<T*>(c->tmp2);
  const T* Sx = pick<T>(dx.fS, dx.dS);
  const T* SxT = pick<T>(dx.fST, dx.dST);
  const T* Sy = pick<T>(dy.fS, dy.dS);
  const T* SyT = pick<T>(dy.fST, dy.dST);
  const double* r = c->zero_buf;
  double* x = c->b[2];
  for (int site = PFD_GS_P1; site <= PFD_GS_P4; ++site) {
    int best = 0;
    for (int cfg = 0; cfg < PFD_GEMM_NCFG && !e; ++cfg) {
      auto run = [&]() -> bool {
        switch (site) {
          case PFD_GS_P1:
            return gemm_launch<T, double, T, 0>(c, cfg, cls, P, r, Ng, Sx, 0, Ny, Nx, Nx, t1, Ng, nullptr, nullptr,
                                         nullptr, nullptr, (const T*)nullptr, 1.0, 0.0);
          case PFD_GS_P2:
            return gemm_launch<T, T, T, 1>(c, cfg, cls, P, SyT, 0, t1, Ng, Ny, Nx, Ny, t2, Ng, dy.dlam, dx.dlam, F.dshift,
                                    nullptr, (const T*)nullptr, 1.0, 0.0);
          case PFD_GS_P3:
            return gemm_launch<T, T, T, 0>(c, cfg, cls, P, Sy, 0, t2, Ng, Ny, Nx, Ny, t1, Ng, nullptr, nullptr, nullptr,
                                    nullptr, (const T*)nullptr, 1.0, 0.0);
          default:
            return gemm_launch<T, T, T, 2>(c, cfg, cls, P, t1, Ng, SxT, 0, Ny, Nx, Nx, (T*)nullptr, Ng, nullptr,
                                    nullptr, nullptr, x, (const T*)nullptr, 1.0, 0.0);
        }
      };
      bool ok = true;
      auto run_ok = [&]() { ok = run(); };
      c->gemm_us[site][ti][cfg] = time_us(c, e0, e1, 5, run_ok, e);
      if (!ok) c->gemm_us[site][ti][cfg] = 0.0;   // not applicable to this shape
      else if (c->gemm_us[site][ti][cfg] < c->gemm_us[site][ti][best]) best = cfg;
    }
    c->gemm_cfg[site][ti] = best;
  }
}

hipError_t autotune(pfd_ctx* c) {
  Family& F = c->fam[PFD_FAM_U];
  Dir1D& dx = c->dirs[F.ix];
  Dir1D& dy = c->dirs[F.iy];
  const bool fp32 = c->prob.precision == PFD_REFINED_FP32;
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e) return e;
  e = hipEventCreate(&e1);
  if (e) { (void)hipEventDestroy(e0); return e; }
  const int saved = c->prof_on;
  c->prof_on = 0;
  {
    // device limits for the LDS-resident pass kernels (k_srp): compute units and the LDS a
    // work-group may take (gfx950: 160 KB, above the default dynamic limit)
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) c->num_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      c->lds_max = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0)
      c->hold_ticks = (long long)v / 2;   // kHz -> ticks in 0.5 ms
    // the single- and multi-instance forms of the LDS-resident pass may take all of the LDS
    bool ok = true;
    for (const void* f : {Kern<k_srp<double, 0>>::single(), Kern<k_srp<double, 0>>::multi(),
                          Kern<k_srp<float, 2>>::single(), Kern<k_srp<float, 2>>::multi(),
                          Kern<k_srp<float, 3>>::single(), Kern<k_srp<float, 3>>::multi()})
      ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, c->lds_max) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      c->lds_max = std::min(c->lds_max, 64 * 1024);
    }
  }
  c->p1_srp = 0;
  c->p4_tg = 0;
  if (fp32)
    tune_fdm_sites<float>(c, e0, e1, e);
  else
    tune_fdm_sites<double>(c, e0, e1, e);
  if (c->is3d && !e) {
    int best = 0;
    for (int cfg = 0; cfg < PFD_GEMM_NCFG && !e; ++cfg) {
      auto run = [&]() -> bool {
        return gemm_launch<double, double, double, 0>(c, cfg, PFD_PROF_ZFFT, 1, c->Wf, 0L, c->zero_buf, 0L, c->planes,
                                               (int)c->Ng, c->planes, c->b[2], 0L, nullptr, nullptr, nullptr,
                                               nullptr, (const double*)nullptr, 1.0, 0.0);
      };
      bool ok = true;
      auto run_ok = [&]() { ok = run(); };
      c->gemm_us[PFD_GS_Z][1][cfg] = time_us(c, e0, e1, 5, run_ok, e);
      if (!ok) c->gemm_us[PFD_GS_Z][1][cfg] = 0.0;
      else if (c->gemm_us[PFD_GS_Z][1][cfg] < c->gemm_us[PFD_GS_Z][1][best]) best = cfg;
    }
    c->gemm_cfg[PFD_GS_Z][1] = best;
    if (c->zlg > 0 && !e) {   // the FFT, for power-of-two plane counts
      const int saved_cfg = c->gemm_cfg[PFD_GS_Z][1];
      c->gemm_cfg[PFD_GS_Z][1] = PFD_ZFFT_CFG;
      auto run = [&]() { ztrans(c, c->Wf, c->zero_buf, c->b[2], nullptr, 1.0, 0.0); };
      c->zfft_us = time_us(c, e0, e1, 5, run, e);
      if (!(c->zfft_us < c->gemm_us[PFD_GS_Z][1][best])) c->gemm_cfg[PFD_GS_Z][1] = saved_cfg;
    }
  }
  for (int v = 0; v < 2 && !e; ++v) {   // residual kernels
    c->resid_variant = v;
    auto run = [&]() { residual(c, PFD_FAM_U, c->zero_buf, c->b[2], c->r, 0, nullptr); };
    c->resid_us[v] = time_us(c, e0, e1, 10, run, e);
  }
  c->resid_variant = (c->resid_us[1] <= c->resid_us[0]) ? 1 : 0;
  auto run_fdm = [&]() {
    if (fp32)
      fdm_correct<float>(c, dx, dy, F.dshift, dx.fS, dx.fST, dy.fS, dy.fST, c->zero_buf, c->b[2]);
    else
      fdm_correct<double>(c, dx, dy, F.dshift, dx.dS, dx.dST, dy.dS, dy.dST, c->zero_buf, c->b[2]);
  };
  for (int v = 0; v < 2 && !e; ++v) {
    c->fdm_variant = v;
    c->fdm_us[v] = time_us(c, e0, e1, 10, run_fdm, e);
  }
  {   // fused middle passes: the column-block width with the faster correction
    c->fdm_variant = 2;
    c->fdm_us[2] = 0.0;
    for (int tn = 1; tn <= 2 && !e; ++tn) {
      const size_t lds = 2 * (fp32 ? 4 : 8) * (size_t)((c->Ny + 15) & ~15) * FDM_MID_LDC(16 * tn);
      if (lds > GEMM_LDS_MAX) continue;
      c->mid_tn = tn;
      c->p4_tg = 0;
      const double us = time_us(c, e0, e1, 10, run_fdm, e);
      if (c->fdm_us[2] == 0.0 || us < c->fdm_us[2]) {
        c->fdm_us[2] = us;
        c->mid_best_tn = tn;
      }
    }
    c->mid_tn = c->mid_best_tn;
    int best_tg = 0;
    const bool srp_ok = srp_lds(c, c->Nx, c->Nx);
    for (const int tg : {1, 6, 2, 3, 4, 5}) {   // the refined last pass: each form of k_p4, k_srp
      if (!fp32 || !(c->fdm_us[2] > 0.0) || e) break;
      if (tg == 5 && !srp_ok) continue;
      c->p4_tg = tg;
      const double us = time_us(c, e0, e1, 10, run_fdm, e);
      if (us < c->fdm_us[2]) {
        c->fdm_us[2] = us;
        best_tg = tg;
      }
    }
    c->p4_tg = best_tg;
  }
  c->fdm_variant = (c->fdm_us[1] <= c->fdm_us[0]) ? 1 : 0;
  if (c->fdm_us[2] > 0.0 && c->fdm_us[2] < c->fdm_us[c->fdm_variant]) c->fdm_variant = 2;
  if (fp32 && c->fdm_variant != 1 && srp_lds(c, c->Nx, c->Nx) && !e) {   // refined first pass with Sx in LDS
    c->p1_srp = 1;
    const double us = time_us(c, e0, e1, 10, run_fdm, e);
    if (us < c->fdm_us[c->fdm_variant]) c->fdm_us[c->fdm_variant] = us;
    else c->p1_srp = 0;
  }
  c->resid_us[2] = 0.0;
  if (fp32 && c->fdm_variant != 1 && !e) {
    // residual fused with the first pass against the separate residual and first-pass GEMM
    float* t1 = reinterpret_cast<float*>(c->tmp);
    bool ok = true;
    auto fused = [&]() {
      ok = res_p1_launch(c, PFD_FAM_U, c->zero_buf, c->b[2], c->fam[PFD_FAM_U].dshift, c->planes, t1, no_chk());
    };
    auto separate = [&]() {
      residual(c, PFD_FAM_U, c->zero_buf, c->b[2], c->r, 0, nullptr);
      gemm<float, double, float, 0>(c, PFD_GS_P1, c->planes, c->r, c->Ng, dx.fS, 0, c->Ny, c->Nx, c->Nx, t1,
                                    c->Ng, nullptr, nullptr, nullptr, nullptr);
    };
    const double us_f = time_us(c, e0, e1, 10, fused, e);
    const double us_s = time_us(c, e0, e1, 10, separate, e);
    if (ok) {
      c->resid_us[2] = us_f;
      if (us_f < us_s) c->resid_variant = 2;
    }
  }
  (void)hipEventDestroy(e0);   // after the last timing that records them
  (void)hipEventDestroy(e1);
  c->prof_on = saved;
  if (!e) e = hipGetLastError();
  return e;
}

// ================================================================== step orchestration
#define FLD(f, lv) c->fld[f][(lv) == 0 ? c->cur : 1 - c->cur]

static void ztrans(pfd_ctx* c, const double* W, const double* in, double* out, const double* in2, double c1,
                   double c2);

hipError_t update_E(pfd_ctx* c) {
  const Geo& g = c->geo;
  dim3 eg(c->geo.nx * c->geo.ny, (c->planes + c->geo.ppw - 1) / c->geo.ppw), eb(((c->geo.ppw * c->nq + 63) / 64) * 64);
  const long tot = (long)c->planes * c->Ng;
  const double* Ez = nullptr;
  if (c->is3d) {
    ztrans(c, c->Wd, c->spec[F_V][c->cur], c->fld[F_EZ][0], nullptr, 1.0, 0.0);
    Ez = c->fld[F_EZ][0];
  }
  Kern<k_E_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, c->stream, g, FLD(F_V, 0), c->Lb[0], c->Lb[1]);
  Kern<k_E_nodal>::launch(c, PFD_PROF_NODAL, dim3(nblk(tot)), dim3(WG), 0, c->stream, g, c->Lb[0], c->Lb[1], c->Mdiag,
                     Ez, c->fld[F_EX][0], c->fld[F_EY][0], c->fld[F_E2][0]);
  return hipGetLastError();
}

// one fixed-point iteration of Remark 3.1 with phi* = phi^n (level 0)
hipError_t potential_iteration(pfd_ctx* c, const double* Vin, double* Vout) {
  Geo g = c->geo;
  Par P = c->par;
  P.cs_n = 1.0;
  P.cs_o = 0.0;
  dim3 eg(g.nx * g.ny, (c->planes + g.ppw - 1) / g.ppw), eb(((g.ppw * c->nq + 63) / 64) * 64);
  const long tot = (long)c->planes * c->Ng;
  const double* ph = FLD(F_PHI, 0);
  Dir1D& dx = c->dirs[c->fam[PFD_FAM_V].ix];
  Dir1D& dy = c->dirs[c->fam[PFD_FAM_V].iy];
  (void)dx;
  (void)dy;
  Kern<k_V_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, c->stream, g, P, ph, ph, Vin, Vin, c->Lb[0]);
  const bool warm = warm_start(c, PFD_FAM_V);
  Kern<k_V_rhs>::launch(c, PFD_PROF_NODAL, dim3(nblk(tot)), dim3(WG), 0, c->stream, g, P, c->lift[PFD_FAM_V], c->Lb[0],
                     c->Mdiag, c->src[PFD_SRC_FV], c->src[PFD_SRC_VD], warm ? Vin : nullptr, Vin, c->b[0], c->r,
                     Vout);
  return solve(c, PFD_FAM_V, c->b[0], Vout, 1, 0, warm ? nullptr : c->r, !warm);
}

hipError_t step_once(pfd_ctx* c, int equilibrium) {
  const Geo& g = c->geo;
  const Par& P = c->par;
  dim3 eg(g.nx * g.ny, (c->planes + g.ppw - 1) / g.ppw), eb(((g.ppw * c->nq + 63) / 64) * 64);
  const long tot = (long)c->planes * c->Ng;
  const dim3 ng(nblk(tot)), nb(WG);
  hipStream_t st = c->stream;
  const int nw = 1 - c->cur;  // level n+1 overwrites level n-1
  // Families refined in FP32 start from the extrapolated history (warm); FP64 solves start from
  // the Dirichlet data with the first residual folded into the right-side kernels (cold)
  auto W = [&](int fam) { return warm_start(c, fam); };
  auto H = [&](int fam, int f, int lv) -> const double* { return W(fam) ? FLD(f, lv) : nullptr; };
  // right sides: b^{n+1} of each family goes to bh[f][nw]; with recycling (refined path, two
  // previous solves recorded) the first residual is formed from bh[f][cur] (= b^n) and b^{n-1}
  auto REC = [&](int fam) { return W(fam) && c->rec_on; };
  auto BB = [&](int f) { return c->bh[f][nw]; };
  auto LR = [&](int f) {
    Lift L = c->lift[f];
    L.bprev = REC(f) ? c->bh[f][c->cur] : nullptr;
    return L;
  };
  auto BP = [&](int f) -> const double* { return REC(f) ? c->bh[f][c->cur] : nullptr; };
  // the solve's first residual, when the right-side kernel formed it (exact when cold)
  auto RR = [&](int f) -> double* { return (!W(f) || REC(f)) ? c->r : nullptr; };
  double* const* S = c->src;
  // ---- V (eq. 54)
  {
    Dir1D& dx = c->dirs[c->fam[PFD_FAM_V].ix];
    Dir1D& dy = c->dirs[c->fam[PFD_FAM_V].iy];
    Kern<k_V_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, FLD(F_PHI, 0), FLD(F_PHI, -1), FLD(F_V, 0), FLD(F_V, -1),
                       c->Lb[0]);
    (void)dx;
    (void)dy;
    Kern<k_V_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_V), c->Lb[0], c->Mdiag, S[PFD_SRC_FV],
                       S[PFD_SRC_VD], H(PFD_FAM_V, F_V, 0), H(PFD_FAM_V, F_V, -1), BB(PFD_FAM_V), c->r,
                       c->fld[F_V][nw]);
    solve(c, PFD_FAM_V, BB(PFD_FAM_V), c->fld[F_V][nw], 1, 0, RR(PFD_FAM_V), !W(PFD_FAM_V));
  }
  // ---- E (eq. 55)
  Kern<k_E_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, c->fld[F_V][nw], c->Lb[0], c->Lb[1]);
  Kern<k_E_nodal>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, c->Lb[0], c->Lb[1], c->Mdiag, (const double*)nullptr,
                     c->fld[F_EX][0], c->fld[F_EY][0], c->fld[F_E2][0]);
  // ---- psi (eq. 56)
  const double* E2 = c->fld[F_E2][0];
  // the equilibrium system (Sec. 2.4) has u = 0: read zeros instead of the velocity
  const double* uxn = equilibrium ? c->zero_buf : FLD(F_UX, 0);
  const double* uxo = equilibrium ? c->zero_buf : FLD(F_UX, -1);
  const double* uyn = equilibrium ? c->zero_buf : FLD(F_UY, 0);
  const double* uyo = equilibrium ? c->zero_buf : FLD(F_UY, -1);
  Kern<k_psi_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, FLD(F_PHI, 0), FLD(F_PHI, -1), uxn, uxo, uyn, uyo, E2,
                     S[PFD_SRC_G], (const double*)nullptr, (const double*)nullptr, (const double*)nullptr, c->Lb[0]);
  Kern<k_psi_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, c->Lb[0], c->bm_open, c->bm_wall, S[PFD_SRC_G1],
                     S[PFD_SRC_G2], S[PFD_SRC_G3], FLD(F_PHI, 0), FLD(F_PHI, -1), E2, H(PFD_FAM_PSI, F_PSI, 0),
                     H(PFD_FAM_PSI, F_PSI, -1), BB(PFD_FAM_PSI), c->U, c->Q2, c->r, c->fld[F_PSI][nw],
                     BP(PFD_FAM_PSI));
  solve(c, PFD_FAM_PSI, BB(PFD_FAM_PSI), c->fld[F_PSI][nw], 1, 0, RR(PFD_FAM_PSI), !W(PFD_FAM_PSI));
  // ---- phi (eq. 57)
  Kern<k_phi_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, c->Mdiag, c->fld[F_PSI][nw], c->bm_open, c->bm_wall,
                     S[PFD_SRC_G2], c->U, H(PFD_FAM_PHI, F_PHI, 0), H(PFD_FAM_PHI, F_PHI, -1), BB(PFD_FAM_PHI),
                     c->r, c->fld[F_PHI][nw], BP(PFD_FAM_PHI));
  solve(c, PFD_FAM_PHI, BB(PFD_FAM_PHI), c->fld[F_PHI][nw], 1, 0, RR(PFD_FAM_PHI), !W(PFD_FAM_PHI));
  if (equilibrium) {
    for (int f : {F_UX, F_UY, F_P}) Kern<k_fill>::launch(c, PFD_PROF_OTHER, ng, nb, 0, st, tot, c->fld[f][nw], 0.0);
  } else {
    // ---- momentum terms, P (eq. 58)
    // phi^{n-1} now holds phi^{n+1}: the momentum kernel takes Q2 (built from phi*) from the psi stage
    Kern<k_mom_elem<false>>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, c->fld[F_PHI][nw], c->fld[F_PSI][nw], E2, c->Q2,
                       FLD(F_UX, 0), FLD(F_UX, -1), FLD(F_UY, 0), FLD(F_UY, -1), FLD(F_P, 0),
                       FLD(F_P, -1), S[PFD_SRC_FX], S[PFD_SRC_FY], c->Lb[0], c->Lb[1], c->Lb[2], Mom3{});
    Kern<k_P_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_P), c->Lb[0], S[PFD_SRC_WX], S[PFD_SRC_WY],
                       S[PFD_SRC_F2], H(PFD_FAM_P, F_P, 0), H(PFD_FAM_P, F_P, -1), BB(PFD_FAM_P), c->r,
                       c->fld[F_P][nw]);
    solve(c, PFD_FAM_P, BB(PFD_FAM_P), c->fld[F_P][nw], 1, 0, RR(PFD_FAM_P), !W(PFD_FAM_P));
    // ---- u (eq. 59)
    Kern<k_gradP_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, c->fld[F_P][nw], (const double*)nullptr, c->Lb[1],
           c->Lb[2], (double*)nullptr);
    Kern<k_u_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_U), c->Lb[1], c->Lb[2], c->bm_open,
                       S[PFD_SRC_F1X], S[PFD_SRC_F1Y], S[PFD_SRC_WX], S[PFD_SRC_WY], H(PFD_FAM_U, F_UX, 0),
                       H(PFD_FAM_U, F_UX, -1), H(PFD_FAM_U, F_UY, 0), H(PFD_FAM_U, F_UY, -1), BB(PFD_FAM_U),
                       BB(PFD_FAM_U) + tot, c->r, c->r + tot, c->fld[F_UX][nw], c->fld[F_UY][nw]);
    // both components as one stack
    solve(c, PFD_FAM_U, BB(PFD_FAM_U), c->fld[F_UX][nw], 2, 0, RR(PFD_FAM_U), !W(PFD_FAM_U));
  }
  Kern<k_check_finite>::launch(c, PFD_PROF_OTHER, dim3(std::min(1024L, (long)nblk(tot))), dim3(WG), 0, st, tot,
         (const double*)c->fld[F_PHI][nw], equilibrium ? (const double*)nullptr : (const double*)c->fld[F_UX][nw],
         c->d_status);
  c->cur = nw;
  return hipGetLastError();
}

// max |a - b| and max |b| over all planes (host result), for the potential fixed point
__device__ __forceinline__ void k_maxdiff_run(const VGrid& vg, long N, const double* a, const double* b,
                                              double* out) {
  __shared__ double s1[WG], s2[WG];
  double m1 = 0.0, m2 = 0.0;
  for (long i = (long)vg.b.x * WG + threadIdx.x; i < N; i += (long)vg.g.x * WG) {
    m1 = fmax(m1, fabs(a[i] - b[i]));
    m2 = fmax(m2, fabs(b[i]));
  }
  s1[threadIdx.x] = m1;
  s2[threadIdx.x] = m2;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + o]);
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * vg.b.x] = s1[0];
    out[2 * vg.b.x + 1] = s2[0];
  }
}
struct k_maxdiff : KDef<&k_maxdiff_run, 0, 0> {};

hipError_t max_abs_diff(pfd_ctx* c, const double* a, const double* b, double* out_host2) {
  const long N = (long)c->planes * c->Ng;
  const int nb = (int)std::min(512L, (long)nblk(N));
  Kern<k_maxdiff>::launch(c, PFD_PROF_OTHER, dim3(nb), dim3(WG), 0, c->stream, N, a, b, c->d_red);
  double h[2 * 512];
  hipMemcpyAsync(h, c->d_red, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, c->stream);
  hipError_t e = hipStreamSynchronize(c->stream);
  out_host2[0] = out_host2[1] = 0.0;
  for (int i = 0; i < nb; ++i) {
    out_host2[0] = fmax(out_host2[0], h[2 * i]);
    out_host2[1] = fmax(out_host2[1], h[2 * i + 1]);
  }
  return e;
}

// ------------------------------------------------------------------ diagnostics
// Block partial sums per instance (vg.b.y) of the quadrature sums behind eq. (14) and the
// mass: q0 int phi, q1 int 1/2 rho |u|^2, q2 phi.(K phi) + int (d_z phi)^2, q3 int (phi^2-1)^2,
// q4 int 1/2 eps |E|^2, q5 wall int phi (phi^2 - 3), q6 max|phi|, q7 non-finite count.
// K phi is the x-y stiffness applied per plane (no mass shift).
__device__ __forceinline__ void k_stats_run(const VGrid& vg, long Ng, long per_inst, Par P,
                                            const double* __restrict__ Mdiag, const double* __restrict__ bw,
                                            const double* __restrict__ phi, const double* __restrict__ ux,
                                            const double* __restrict__ uy, const double* __restrict__ uz,
                                            const double* __restrict__ Ex, const double* __restrict__ Ey,
                                            const double* __restrict__ Ez, const double* __restrict__ Kphi,
                                            const double* __restrict__ dzphi, double* __restrict__ part) {
  __shared__ double red[8][WG];
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long base = (long)vg.b.y * per_inst;
  for (long i = (long)vg.b.x * WG + threadIdx.x; i < per_inst; i += (long)vg.g.x * WG) {
    const long id = base + i;
    const long node = id % Ng;
    const double w = Mdiag[node], p = phi[id];
    double u2 = ux[id] * ux[id] + uy[id] * uy[id];
    double e2 = Ex[id] * Ex[id] + Ey[id] * Ey[id];
    if (uz) u2 += uz[id] * uz[id];
    if (Ez) e2 += Ez[id] * Ez[id];
    const double rho = 0.5 * (P.rho1 + P.rho2) + 0.5 * (P.rho1 - P.rho2) * p;
    const double dw = p * p - 1.0;
    s[0] += w * p;
    s[1] += 0.5 * w * rho * u2;
    s[2] += p * Kphi[id];
    if (dzphi) s[2] += w * dzphi[id] * dzphi[id];
    s[3] += w * dw * dw;
    s[4] += 0.5 * w * eps_of(P, p) * e2;
    s[5] += bw[node] * p * (p * p - 3.0);
    s[6] = fmax(s[6], fabs(p));
    if (!isfinite(p) || !isfinite(u2) || !isfinite(e2)) s[7] += 1.0;
  }
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 8; ++q)
        red[q][threadIdx.x] = (q == 6) ? fmax(red[q][threadIdx.x], red[q][threadIdx.x + o])
                                       : red[q][threadIdx.x] + red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 8) part[((long)vg.b.y * vg.g.x + vg.b.x) * 8 + threadIdx.x] = red[threadIdx.x][0];
}
struct k_stats : KDef<&k_stats_run, 0, 0> {};

hipError_t stats(pfd_ctx* c, double* out) {
  const long tot = (long)c->planes * c->Ng;
  const int ninst = c->is3d ? 1 : c->planes;
  const long per = tot / ninst;
  const int nb = PFD_STAT_NB;
  const int cu = c->cur;
  const double* phi = c->fld[F_PHI][cu];
  double* Kphi = c->r;
  double* dzphi = c->is3d ? c->r + tot : nullptr;
  residual(c, PFD_FAM_PSI, nullptr, phi, Kphi, 1, nullptr, c->zero_buf);
  if (c->is3d) ztrans(c, c->Dz, phi, dzphi, nullptr, 1.0, 0.0);
  Kern<k_stats>::launch(c, PFD_PROF_OTHER, dim3(nb, ninst), dim3(WG), 0, c->stream, c->Ng, per, c->par, c->Mdiag,
         c->bm_wall, phi, c->fld[F_UX][cu], c->fld[F_UY][cu], c->is3d ? c->fld[F_UZ][cu] : nullptr,
         c->fld[F_EX][0], c->fld[F_EY][0], c->is3d ? c->fld[F_EZ][0] : nullptr, Kphi, dzphi, c->d_stats);
  std::vector<double> h((size_t)ninst * nb * 8);
  hipError_t e = hipMemcpyAsync(h.data(), c->d_stats, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) return e;
  const Par& P = c->par;
  const double wz = c->is3d ? c->prob.mesh.lz / c->planes : 1.0;
  const double sigma = 2.0 * std::sqrt(2.0) * P.lam / (3.0 * P.eta);
  for (int i = 0; i < ninst; ++i) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
      for (int q = 0; q < 8; ++q) {
        const double v = h[((size_t)i * nb + b) * 8 + q];
        s[q] = (q == 6) ? std::fmax(s[q], v) : s[q] + v;
      }
    double* o = out + (size_t)i * 8;
    o[0] = s[0] * wz;
    o[1] = s[1] * wz;
    o[2] = (0.5 * P.lam * s[2] + P.lam / (4.0 * P.eta * P.eta) * s[3]) * wz;
    o[3] = s[4] * wz;
    o[4] = sigma * P.cos_theta * 0.25 * s[5] * wz;
    o[5] = o[1] + o[2] + o[3] + o[4];
    o[6] = s[6];
    o[7] = s[7];
  }
  return hipSuccess;
}

// ============================================================ 3D: Fourier in z (Algorithm 2)
// Physical fields are z planes; spectral fields use the packed real layout on the same
// planes: plane 0 = Re k=0, plane 1 = Re k=Nz/2, planes 2k / 2k+1 = Re / Im of mode k.
// The z transforms are the dense packed DFT matrices (Nz x Nz) applied with the batched MFMA
// GEMM: Wf (forward, 1/Nz normalised), Wi (inverse), Wd (spectral -> physical d/dz, i beta_k;
// the Nyquist derivative is 0), Dz = Wd Wf (physical d/dz).

// right side of the per-mode weak forms from the transformed parts:
//   b = scale * (A + i beta_k B)   (bmode 0)   or   scale * (A + beta_k^2 B)   (bmode 1)
//       + mc * M * Cv   (optional spectral term),
// then the initial guess / first residual as in rhs_out (gD, Fn, Fo spectral)
__device__ __forceinline__ void k_spec_rhs_run(const VGrid& vg, Geo g, Par P, Lift L, const double* A,
                                               const double* B, int bmode, double scale, const double* Cv, double mc,
                                               const double* Mdiag, const double* beta2, const double* betad,
                                               const double* gD, const double* Fn, const double* Fo, double* bb,
                                               double* r, double* x0) {
  NODAL_PROLOGUE
  double v = A[id];
  if (B) {
    if (bmode == 0) {
      // the partner plane of a (cos, sin) pair; planes 0 and 1 have beta = 0 and read their
      // neighbour only to add a zero, so the load waits behind no test of beta
      const double bd = betad[pl];
      const double bp = B[((pl & 1) == 0) ? id + g.Ng : id - g.Ng];
      v += ((pl & 1) == 0) ? -bd * bp : bd * bp;
    } else {
      v += beta2[pl] * B[id];
    }
  }
  v *= scale;
  if (Cv) v += mc * Mdiag[node] * Cv[id];
  rhs_out(g, P, L, gD, Fn, Fo, id, (long)pl * g.Ng, ix, iy, v, bb, r, x0);
}
struct k_spec_rhs : KDef<&k_spec_rhs_run, 0, 0> {};

// V: A = DSS(L0) - M f_V,  B = M (eps(phi*) - eps0) d(V*)/dz
__device__ __forceinline__ void k_V_rhs3_run(const VGrid& vg, Geo g, Par P, const double* L0, const double* Mdiag,
                                             const double* fV, const double* phn, const double* pho,
                                             const double* dzV, double* A, double* B) {
  NODAL_PROLOGUE
  A[id] = dss(g, L0, pl, ix, iy) - Mdiag[node] * fV[id];
  const double phs = P.cs_n * phn[id] + P.cs_o * pho[id];
  B[id] = Mdiag[node] * (eps_of(P, phs) - P.eps0) * dzV[id];
}
struct k_V_rhs3 : KDef<&k_V_rhs3_run, 0, 0> {};

// psi: A = DSS(L0) + Bo (g1 + c_psi g2) + Bs (g1 + c_psi U),  B = M Q2 ; U, Q2 kept
__device__ __forceinline__ void k_psi_rhs3_run(const VGrid& vg, Geo g, Par P, const double* L0, const double* Mdiag,
                                               const double* bmo, const double* bmw, const double* g1,
                                               const double* g2, const double* g3, const double* phn,
                                               const double* pho, const double* E2, double* A, double* B, double* U,
                                               double* Q2) {
  NODAL_PROLOGUE
  const double phs = P.cs_n * phn[id] + P.cs_o * pho[id];
  const double u = -g3[id] - thp_of(P, phs);
  U[id] = u;
  const double q2 = h_of(P, phs) - P.S / (P.eta * P.eta) * phs - deps_of(P, phs) * E2[id] / (2.0 * P.lam);
  Q2[id] = q2;
  A[id] = dss(g, L0, pl, ix, iy) + bmo[node] * (g1[id] + P.c_psi * g2[id]) + bmw[node] * (g1[id] + P.c_psi * u);
  B[id] = Mdiag[node] * q2;
}
struct k_psi_rhs3 : KDef<&k_psi_rhs3_run, 0, 0> {};

// phi: boundary part Bo g2 + Bs U (the -M psi part is added in spectral space)
__device__ __forceinline__ void k_phi_bnd3_run(const VGrid& vg, Geo g, const double* bmo, const double* bmw,
                                               const double* g2, const double* U, double* A) {
  NODAL_PROLOGUE
  A[id] = bmo[node] * g2[id] + bmw[node] * U[id];
}
struct k_phi_bnd3 : KDef<&k_phi_bnd3_run, 0, 0> {};

// Phi_hat = psi_hat - c_psi phi_hat - Q2_hat, with Q2_hat = (M Q2)_hat / M (reading R-J)
__device__ __forceinline__ void k_Phi_hat3_run(const VGrid& vg, Geo g, Par P, const double* psh, const double* phh,
                                               const double* BQ, const double* Mdiag, double* out) {
  NODAL_PROLOGUE
  out[id] = psh[id] - P.c_psi * phh[id] - BQ[id] / Mdiag[node];
}
struct k_Phi_hat3 : KDef<&k_Phi_hat3_run, 0, 0> {};

// P: A = DSS(L0) - rho0 gamma0/dt sum_walls int (n.w) q,  B = DSS(LBP)
__device__ __forceinline__ void k_P_rhs3_run(const VGrid& vg, Geo g, Par P, const double* L0, const double* LBP,
                                             const double* wx, const double* wy, double* A, double* B) {
  NODAL_PROLOGUE
  double v = dss(g, L0, pl, ix, iy);
  const double c = P.rho0 * P.gamma0 / P.dt;
  const double nw[4] = {-wy[id], wy[id], -wx[id], wx[id]};
  for (int sd = 0; sd < 4; ++sd)
    if (g.side_type[sd] == PFD_WALL) v -= c * g.bm_side[sd][node] * nw[sd];
  A[id] = v;
  B[id] = dss(g, LBP, pl, ix, iy);
}
struct k_P_rhs3 : KDef<&k_P_rhs3_run, 0, 0> {};

// u: A_x, B_x, A_y, B_y, A_z (open-side f1 added to the A parts)
__device__ __forceinline__ void k_u_rhs3_run(const VGrid& vg, Geo g, const double* L1, const double* LBx,
                                             const double* L2, const double* LBy, const double* LAz,
                                             const double* bmo, const double* f1x, const double* f1y,
                                             const double* f1z, double* Ax, double* Bx, double* Ay, double* By,
                                             double* Az) {
  NODAL_PROLOGUE
  Ax[id] = dss(g, L1, pl, ix, iy) + bmo[node] * f1x[id];
  Bx[id] = dss(g, LBx, pl, ix, iy);
  Ay[id] = dss(g, L2, pl, ix, iy) + bmo[node] * f1y[id];
  By[id] = dss(g, LBy, pl, ix, iy);
  Az[id] = dss(g, LAz, pl, ix, iy) + bmo[node] * f1z[id];
}
struct k_u_rhs3 : KDef<&k_u_rhs3_run, 0, 0> {};

// ------------------------------------------------------------------ FFT along z
// Batched real FFT along z for a power-of-two number of planes Nz = 4..256 (the dense-DFT GEMM
// above covers any even count).  Two real node columns a, b travel as one complex sequence
// z = f_a + i f_b; the length-Nz transform is split as Nz = N1 N2 (four-step / Cooley-Tukey
// with one LDS exchange): a thread holds N1 samples z_{n2 + N2 n1} in registers and transforms
// over n1, multiplies by exp(-2 pi i n2 k1 / Nz), and after the LDS exchange a thread transforms
// the N2 values of one k1 over n2, giving c_{k1 + N1 k2}.  The inverse runs the same steps in
// the mirrored order.  The spectra of the two real columns are separated with
// C_a = (Z_k + conj Z_{Nz-k}) / 2, C_b = (Z_k - conj Z_{Nz-k}) / 2i, and joined again as
// Z = C_a + i C_b for the inverse.  Modes (same results as the packed DFT matrices up to
// rounding):
//   0  forward   f -> packed spectrum / Nz            (Wf)
//   1  inverse   packed spectrum -> f                 (Wi)
//   2  d/dz of a packed spectrum -> physical          (Wd: i beta_k, k = 0 and Nyquist -> 0)
//   3  physical d/dz: forward, i beta_k, inverse      (Dz)
// Packed layout: plane 0 = Re c_0, plane 1 = Re c_{Nz/2}, planes 2k, 2k+1 = Re, Im c_k.
// Multiplying by i beta(k) with beta odd in k (beta(Nz-k) = -beta(k)) keeps Z = C_a + i C_b
// consistent, so modes 2 and 3 apply it to Z directly.  One launch runs up to ZB_MAX
// independent transforms (vg.b.y), each with its own mode, input and output.
template <int N>
struct ZLog2 {
  static constexpr int v = 1 + ZLog2<N / 2>::v;
};
template <>
struct ZLog2<1> {
  static constexpr int v = 0;
};

// in-register DFT of length N (radix-2, decimation in time, natural order in and out):
// x_j <- sum_i x_i w^{+-ij}, w = exp(-2 pi i / N), twiddles W_Nz^m = (wr[m], wi[m]) from LDS
template <int N, int NZ, bool INV>
__device__ __forceinline__ void zdft_reg(double (&re)[N], double (&im)[N], const double* wr, const double* wi) {
  constexpr int L = ZLog2<N>::v;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    int r = 0;
#pragma unroll
    for (int bit = 0; bit < L; ++bit) r |= ((i >> bit) & 1) << (L - 1 - bit);
    if (i < r) {
      const double tr = re[i], ti = im[i];
      re[i] = re[r];
      im[i] = im[r];
      re[r] = tr;
      im[r] = ti;
    }
  }
#pragma unroll
  for (int s = 0; s < L; ++s) {
    const int m = 1 << s;
#pragma unroll
    for (int g = 0; g < N; g += 2 * m)
#pragma unroll
      for (int p = 0; p < m; ++p) {
        const int a = g + p, b = a + m;
        double xr = re[b], xi = im[b];
        if (p != 0) {
          const int tw = p * (NZ / (2 * m));
          const double c = wr[tw], sn = INV ? -wi[tw] : wi[tw];
          const double yr = c * xr - sn * xi;
          xi = c * xi + sn * xr;
          xr = yr;
        }
        re[b] = re[a] - xr;
        im[b] = im[a] - xi;
        re[a] += xr;
        im[a] += xi;
      }
  }
}

// i beta(k) as a multiplier of Z_k (0 for k = 0 and the Nyquist mode)
template <int NZ>
__device__ __forceinline__ double zbeta(int k, const double* __restrict__ betad) {
  const bool lo = k < NZ / 2;
  const int kk = lo ? k : NZ - k;
  const double b = betad[2 * (kk < NZ / 2 ? kk : 0)];
  return (k == 0 || k == NZ / 2) ? 0.0 : (lo ? b : -b);
}

// work-group: P column pairs (nodes n0 + c and n0 + P + c), T = P N2 threads; thread t owns
// column c = t % P and row t / P (n2 in the first half-transform, k1 = t / P + N2 r in the second)
template <int LG>
struct ZfftShape {
  static constexpr int NZ = 1 << LG, N1 = 1 << ((LG + 1) / 2), N2 = 1 << (LG / 2);
  static constexpr int P = (4096 / NZ) < 64 ? (4096 / NZ) : 64;
  static constexpr int T = P * N2;
  static constexpr int RS = N2 * P + P;   // LDS stride between k1 rows (padded)
};

#define ZB_MAX 6
struct ZBatch {
  const double* in[ZB_MAX];
  const double* in2[ZB_MAX];   // second input (c1 in + c2 in2) when the kernel is built for it
  double* out[ZB_MAX];
  int mode[ZB_MAX];
};

template <int LG, bool TWO>
__device__ __forceinline__ void k_zfft_run(const VGrid& vg, ZBatch zb, long Ng, double c1, double c2,
                                           const double* __restrict__ twr_g, const double* __restrict__ twi_g,
                                           const double* __restrict__ betad) {
  using S = ZfftShape<LG>;
  constexpr int NZ = S::NZ, N1 = S::N1, N2 = S::N2, P = S::P, T = S::T, RS = S::RS;
  __shared__ double lr[N1 * RS], li[N1 * RS], wr[NZ], wi[NZ];
  const int e = vg.b.y;
  const int mode = zb.mode[e];
  const double* __restrict__ in = zb.in[e];
  const double* __restrict__ in2 = zb.in2[e];
  double* __restrict__ out = zb.out[e];
  const int t = threadIdx.x;
  for (int m = t; m < NZ; m += T) {   // W_Nz^m for m = 0..Nz-1 from the half table
    const bool lo = m <= NZ / 2;
    const int mm = lo ? m : NZ - m;
    wr[m] = twr_g[mm];
    wi[m] = lo ? twi_g[mm] : -twi_g[mm];
  }
  const int c = t % P, row = t / P;
  const long n0 = (long)vg.b.x * (2 * P);
  const long na = n0 + c, nb = n0 + P + c;
  const bool va = na < Ng, vb = nb < Ng;
  const long ia = va ? na : 0, ib = vb ? nb : 0;   // clamped addresses, values masked after the load
  // the N1 input planes row + N2 q of both columns (coalesced along the nodes)
  double xr[N1], xi[N1];
#pragma unroll
  for (int q = 0; q < N1; ++q) {
    const long o = (long)(row + N2 * q) * Ng;
    double u = in[o + ia], v = in[o + ib];
    if (TWO) {
      u = c1 * u + c2 * in2[o + ia];
      v = c1 * v + c2 * in2[o + ib];
    }
    xr[q] = va ? u : 0.0;
    xi[q] = vb ? v : 0.0;
  }
  __syncthreads();   // twiddle table

  if (mode == 0 || mode == 3) {
    // first half: n2 = row, transform over n1
    zdft_reg<N1, NZ, false>(xr, xi, wr, wi);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      const int tw = row * k1;
      const double cr = wr[tw], ci = wi[tw];
      lr[k1 * RS + row * P + c] = cr * xr[k1] - ci * xi[k1];
      li[k1 * RS + row * P + c] = cr * xi[k1] + ci * xr[k1];
    }
    __syncthreads();
    // second half: k1 = row + N2 r, transform over n2
#pragma unroll
    for (int r = 0; r < N1 / N2; ++r) {
      const int k1 = row + N2 * r;
      double yr[N2], yi[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) {
        yr[n2] = lr[k1 * RS + n2 * P + c];
        yi[n2] = li[k1 * RS + n2 * P + c];
      }
      zdft_reg<N2, NZ, false>(yr, yi, wr, wi);
      if (mode == 3) {   // i beta(k) / Nz, then back over k2 and the conjugate twiddle
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const double b = zbeta<NZ>(k1 + N1 * k2, betad) * (1.0 / NZ);
          const double zr = yr[k2];
          yr[k2] = -b * yi[k2];
          yi[k2] = b * zr;
        }
        zdft_reg<N2, NZ, true>(yr, yi, wr, wi);
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
          const int tw = n2 * k1;
          const double cr = wr[tw], ci = -wi[tw];
          const double ur = cr * yr[n2] - ci * yi[n2], ui = cr * yi[n2] + ci * yr[n2];
          yr[n2] = ur;
          yi[n2] = ui;
        }
      }
#pragma unroll
      for (int j = 0; j < N2; ++j) {   // same LDS slots as read (k2 slots for mode 0)
        lr[k1 * RS + j * P + c] = yr[j];
        li[k1 * RS + j * P + c] = yi[j];
      }
    }
    __syncthreads();
    if (mode == 0) {
      // packed output plane p = row + N2 q, separated spectra of columns a (real) and b (imag)
      constexpr double sc = 1.0 / NZ;
#pragma unroll
      for (int q = 0; q < N1; ++q) {
        const int p = row + N2 * q;
        const int k = p == 0 ? 0 : (p == 1 ? NZ / 2 : (p >> 1));
        const int km = (NZ - k) & (NZ - 1);
        const int sk = (k % N1) * RS + (k / N1) * P + c, sm = (km % N1) * RS + (km / N1) * P + c;
        const double zr = lr[sk], zi = li[sk], mr = lr[sm], mi = li[sm];
        const bool imag = p >= 2 && (p & 1);
        const double oa = imag ? 0.5 * (zi - mi) : 0.5 * (zr + mr);
        const double ob = imag ? 0.5 * (mr - zr) : 0.5 * (zi + mi);
        if (va) out[(long)p * Ng + na] = sc * oa;
        if (vb) out[(long)p * Ng + nb] = sc * ob;
      }
      return;
    }
  } else {
    // modes 1, 2: packed planes staged in LDS (plane p of column a at lr[p P + c], of b at li),
    // then Z_k = C_a(k) + i C_b(k) with the Hermitian completion for k > Nz/2
#pragma unroll
    for (int q = 0; q < N1; ++q) {
      lr[(row + N2 * q) * P + c] = xr[q];
      li[(row + N2 * q) * P + c] = xi[q];
    }
    __syncthreads();
    double zr_[N1], zi_[N1];   // Z for k1 = row + N2 r, k2: index r N2 + k2
#pragma unroll
    for (int r = 0; r < N1 / N2; ++r) {
      const int k1 = row + N2 * r;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int k = k1 + N1 * k2;
        const bool lo = k <= NZ / 2;
        const int kk = lo ? k : NZ - k;
        const bool cplx = kk != 0 && kk != NZ / 2;
        const int pre = kk == 0 ? 0 : (kk == NZ / 2 ? 1 : 2 * kk), pim = cplx ? 2 * kk + 1 : 0;
        const double sg = lo ? 1.0 : -1.0;
        const double Ar = lr[pre * P + c], Br = li[pre * P + c];
        const double Ai = cplx ? sg * lr[pim * P + c] : 0.0, Bi = cplx ? sg * li[pim * P + c] : 0.0;
        double zr = Ar - Bi, zi = Ai + Br;
        if (mode == 2) {
          const double b = zbeta<NZ>(k, betad);
          const double tr = zr;
          zr = -b * zi;
          zi = b * tr;
        }
        zr_[r * N2 + k2] = zr;
        zi_[r * N2 + k2] = zi;
      }
    }
    __syncthreads();   // staging read before the slots are reused
#pragma unroll
    for (int r = 0; r < N1 / N2; ++r) {
      const int k1 = row + N2 * r;
      double yr[N2], yi[N2];
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        yr[k2] = zr_[r * N2 + k2];
        yi[k2] = zi_[r * N2 + k2];
      }
      zdft_reg<N2, NZ, true>(yr, yi, wr, wi);
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) {
        const int tw = n2 * k1;
        const double cr = wr[tw], ci = -wi[tw];
        lr[k1 * RS + n2 * P + c] = cr * yr[n2] - ci * yi[n2];
        li[k1 * RS + n2 * P + c] = cr * yi[n2] + ci * yr[n2];
      }
    }
    __syncthreads();
  }
  // last half of the inverse: n2 = row, transform over k1, z_{n2 + N2 n1} = f_a + i f_b
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    xr[k1] = lr[k1 * RS + row * P + c];
    xi[k1] = li[k1 * RS + row * P + c];
  }
  zdft_reg<N1, NZ, true>(xr, xi, wr, wi);
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
    const long z = row + N2 * n1;
    if (va) out[z * Ng + na] = xr[n1];
    if (vb) out[z * Ng + nb] = xi[n1];
  }
}
template <int LG, bool TWO>
struct k_zfft : KDef<&k_zfft_run<LG, TWO>, ZfftShape<LG>::T, 0> {};

template <int LG>
static void zfft_launch(pfd_ctx* c, const ZBatch& zb, int n, bool two, double c1, double c2) {
  using S = ZfftShape<LG>;
  const dim3 grid((unsigned)((c->Ng + 2 * S::P - 1) / (2 * S::P)), (unsigned)n);
  if (two)
    Kern<k_zfft<LG, true>>::launch(c, PFD_PROF_ZFFT, grid, dim3(S::T), 0, c->stream, zb, c->Ng, c1, c2, c->twr, c->twi,
           c->d_betad);
  else
    Kern<k_zfft<LG, false>>::launch(c, PFD_PROF_ZFFT, grid, dim3(S::T), 0, c->stream, zb, c->Ng, c1, c2, c->twr, c->twi,
           c->d_betad);
}

// out = W in  (or W (c1 in + c2 in2)) along z for every node: one GEMM, M = K = Nz, N = Ng
static void ztrans(pfd_ctx* c, const double* W, const double* in, double* out, const double* in2 = nullptr,
                   double c1 = 1.0, double c2 = 0.0);
// n independent z transforms (n <= ZB_MAX), each W[i] in[i] (or W[i] (c1 in[i] + c2 in2[i]));
// in2 is given for all of them or for none.  The FFT runs them as one launch.
static void ztrans_n(pfd_ctx* c, int n, const double* const* W, const double* const* in, double* const* out,
                     const double* const* in2 = nullptr, double c1 = 1.0, double c2 = 0.0) {
  if (c->gemm_cfg[PFD_GS_Z][1] == PFD_ZFFT_CFG && c->zlg > 0 && n >= 1 && n <= ZB_MAX) {
    ZBatch zb{};
    for (int i = 0; i < n; ++i) {
      zb.mode[i] = (W[i] == c->Wf) ? 0 : (W[i] == c->Wi) ? 1 : (W[i] == c->Wd) ? 2 : 3;
      zb.in[i] = in[i];
      zb.in2[i] = in2 ? in2[i] : in[i];
      zb.out[i] = out[i];
    }
    const bool two = in2 != nullptr;
    switch (c->zlg) {
      case 2: zfft_launch<2>(c, zb, n, two, c1, c2); return;
      case 3: zfft_launch<3>(c, zb, n, two, c1, c2); return;
      case 4: zfft_launch<4>(c, zb, n, two, c1, c2); return;
      case 5: zfft_launch<5>(c, zb, n, two, c1, c2); return;
      case 6: zfft_launch<6>(c, zb, n, two, c1, c2); return;
      case 7: zfft_launch<7>(c, zb, n, two, c1, c2); return;
      case 8: zfft_launch<8>(c, zb, n, two, c1, c2); return;
      default: break;   // not reached: zlg is set for 4 <= Nz <= 256 only
    }
  }
  for (int i = 0; i < n; ++i) {
    const double* b2 = in2 ? in2[i] : nullptr;
    if (!gemm_launch<double, double, double, 0>(c, c->gemm_cfg[PFD_GS_Z][1], PFD_PROF_ZFFT, 1, W[i], 0L, in[i], 0L,
                                                c->planes, (int)c->Ng, c->planes, out[i], 0L, nullptr, nullptr,
                                                nullptr, nullptr, b2, c1, c2))
      gemm_launch<double, double, double, 0>(c, 0, PFD_PROF_ZFFT, 1, W[i], 0L, in[i], 0L, c->planes, (int)c->Ng,
                                             c->planes, out[i], 0L, nullptr, nullptr, nullptr, nullptr, b2, c1, c2);
  }
}
static void ztrans(pfd_ctx* c, const double* W, const double* in, double* out, const double* in2, double c1,
                   double c2) {
  ztrans_n(c, 1, &W, &in, &out, in2 ? &in2 : nullptr, c1, c2);
}

// spectral copies of the Dirichlet sources that changed since the last step (reading R-dir3d)
void refresh_spectral_sources(pfd_ctx* c) {
  const int ids[5] = {PFD_SRC_VD, PFD_SRC_F2, PFD_SRC_WX, PFD_SRC_WY, PFD_SRC_WZ};
  for (int s : ids)
    if (c->src_dirty[s]) {
      ztrans(c, c->Wf, c->src[s], c->srcS[s]);
      c->src_dirty[s] = 0;
    }
}

#define SPEC(f, lv) c->spec[f][(lv) == 0 ? c->cur : 1 - c->cur]

hipError_t step_once_3d(pfd_ctx* c, int equilibrium) {
  const Geo& g = c->geo;
  const Par& P = c->par;
  dim3 eg(g.nx * g.ny, (c->planes + g.ppw - 1) / g.ppw), eb(((g.ppw * c->nq + 63) / 64) * 64);
  const long tot = (long)c->planes * c->Ng;
  const dim3 ng(nblk(tot)), nb(WG);
  hipStream_t st = c->stream;
  const int nw = 1 - c->cur;
  auto W = [&](int fam) { return warm_start(c, fam); };
  auto H = [&](int fam, int f, int lv) -> const double* { return W(fam) ? SPEC(f, lv) : nullptr; };
  // right sides per family and level, recycled for the refined path's first residual (as in 2D)
  auto REC = [&](int fam) { return W(fam) && c->rec_on; };
  auto BB = [&](int f) { return c->bh[f][nw]; };
  auto LR = [&](int f, int comp) {
    Lift L = c->lift[f];
    L.bprev = REC(f) ? c->bh[f][c->cur] + comp * tot : nullptr;
    return L;
  };
  auto RR = [&](int f) -> double* { return (!W(f) || REC(f)) ? c->r : nullptr; };
  double* const* S = c->src;
  double **ph = c->ph, **sp = c->sp, **dz = c->dz, **Lb = c->Lb;
  refresh_spectral_sources(c);
  {
    // z-derivatives of the extrapolated V, phi (and u, P) in one launch: dz[0..5]
    const double* Ws[6] = {c->Wd, c->Wd, c->Wd, c->Wd, c->Wd, c->Wd};
    const double* ins[6] = {SPEC(F_V, 0), SPEC(F_PHI, 0), nullptr, nullptr, nullptr, nullptr};
    const double* olds[6] = {SPEC(F_V, -1), SPEC(F_PHI, -1), nullptr, nullptr, nullptr, nullptr};
    if (!equilibrium) {
      const int fs[4] = {F_UX, F_UY, F_UZ, F_P};
      for (int i = 0; i < 4; ++i) {
        ins[2 + i] = SPEC(fs[i], 0);
        olds[2 + i] = SPEC(fs[i], -1);
      }
    }
    ztrans_n(c, equilibrium ? 2 : 6, Ws, ins, dz, olds, P.cs_n, P.cs_o);
  }
  // ---- V (eq. 74)
  Kern<k_V_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, FLD(F_PHI, 0), FLD(F_PHI, -1), FLD(F_V, 0), FLD(F_V, -1),
         Lb[0]);
  Kern<k_V_rhs3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, Lb[0], c->Mdiag, S[PFD_SRC_FV], FLD(F_PHI, 0),
         FLD(F_PHI, -1), dz[0], ph[0], ph[1]);
  const double* Wff[5] = {c->Wf, c->Wf, c->Wf, c->Wf, c->Wf};
  const double* Wfi[3] = {c->Wi, c->Wi, c->Wi};
  const double* Wid[2] = {c->Wi, c->Wd};
  const double* ph01[2] = {ph[0], ph[1]};
  ztrans_n(c, 2, Wff, ph01, sp);
  Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_V, 0), sp[0], sp[1], 0, 1.0 / P.eps0,
         (const double*)nullptr, 0.0, c->Mdiag, c->d_beta2, c->d_betad, c->srcS[PFD_SRC_VD], H(PFD_FAM_V, F_V, 0),
         H(PFD_FAM_V, F_V, -1), BB(PFD_FAM_V), c->r, c->spec[F_V][nw]);
  solve(c, PFD_FAM_V, BB(PFD_FAM_V), c->spec[F_V][nw], 1, 0, RR(PFD_FAM_V), !W(PFD_FAM_V));
  {
    // V and E_z = i beta V (reading R-Ez) from the new spectrum in one launch
    const double* ins[2] = {c->spec[F_V][nw], c->spec[F_V][nw]};
    double* outs[2] = {c->fld[F_V][nw], c->fld[F_EZ][0]};
    ztrans_n(c, 2, Wid, ins, outs);
  }
  // ---- E (eq. 78): E_x, E_y by plane-wise projection
  Kern<k_E_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, c->fld[F_V][nw], Lb[0], Lb[1]);
  Kern<k_E_nodal>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, Lb[0], Lb[1], c->Mdiag, (const double*)c->fld[F_EZ][0],
         c->fld[F_EX][0], c->fld[F_EY][0], c->fld[F_E2][0]);
  const double* E2 = c->fld[F_E2][0];
  // ---- psi (eq. 75)
  const double* uxn = equilibrium ? c->zero_buf : FLD(F_UX, 0);
  const double* uxo = equilibrium ? c->zero_buf : FLD(F_UX, -1);
  const double* uyn = equilibrium ? c->zero_buf : FLD(F_UY, 0);
  const double* uyo = equilibrium ? c->zero_buf : FLD(F_UY, -1);
  const double* uzn = equilibrium ? c->zero_buf : FLD(F_UZ, 0);
  const double* uzo = equilibrium ? c->zero_buf : FLD(F_UZ, -1);
  Kern<k_psi_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, FLD(F_PHI, 0), FLD(F_PHI, -1), uxn, uxo, uyn, uyo, E2,
         S[PFD_SRC_G], uzn, uzo, (const double*)dz[1], Lb[0]);
  Kern<k_psi_rhs3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, Lb[0], c->Mdiag, c->bm_open, c->bm_wall, S[PFD_SRC_G1],
         S[PFD_SRC_G2], S[PFD_SRC_G3], FLD(F_PHI, 0), FLD(F_PHI, -1), E2, ph[0], ph[1], c->U, c->Q2);
  ztrans_n(c, 2, Wff, ph01, sp);  // sp[1] = (M Q2)_hat, kept for Phi_hat below
  Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_PSI, 0), sp[0], sp[1], 1, 1.0,
         (const double*)nullptr, 0.0, c->Mdiag, c->d_beta2, c->d_betad, (const double*)nullptr,
         H(PFD_FAM_PSI, F_PSI, 0), H(PFD_FAM_PSI, F_PSI, -1), BB(PFD_FAM_PSI), c->r, c->spec[F_PSI][nw]);
  solve(c, PFD_FAM_PSI, BB(PFD_FAM_PSI), c->spec[F_PSI][nw], 1, 0, RR(PFD_FAM_PSI), !W(PFD_FAM_PSI));
  ztrans(c, c->Wi, c->spec[F_PSI][nw], c->fld[F_PSI][nw]);
  // ---- phi (eq. 76, reading R-psi)
  Kern<k_phi_bnd3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, c->bm_open, c->bm_wall, S[PFD_SRC_G2], c->U, ph[0]);
  ztrans(c, c->Wf, ph[0], sp[0]);
  Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_PHI, 0), sp[0], (const double*)nullptr, 0,
         1.0, (const double*)c->spec[F_PSI][nw], -1.0, c->Mdiag, c->d_beta2, c->d_betad, (const double*)nullptr,
         H(PFD_FAM_PHI, F_PHI, 0), H(PFD_FAM_PHI, F_PHI, -1), BB(PFD_FAM_PHI), c->r, c->spec[F_PHI][nw]);
  solve(c, PFD_FAM_PHI, BB(PFD_FAM_PHI), c->spec[F_PHI][nw], 1, 0, RR(PFD_FAM_PHI), !W(PFD_FAM_PHI));
  {
    // phi, and its z-derivative for the momentum terms
    const double* ins[2] = {c->spec[F_PHI][nw], c->spec[F_PHI][nw]};
    double* outs[2] = {c->fld[F_PHI][nw], dz[0]};
    ztrans_n(c, equilibrium ? 1 : 2, Wid, ins, outs);
  }
  if (equilibrium) {
    for (int f : {F_UX, F_UY, F_UZ, F_P}) {
      Kern<k_fill>::launch(c, PFD_PROF_OTHER, ng, nb, 0, st, tot, c->fld[f][nw], 0.0);
      Kern<k_fill>::launch(c, PFD_PROF_OTHER, ng, nb, 0, st, tot, c->spec[f][nw], 0.0);
    }
  } else {
    // ---- momentum terms (eq. 49 and the G, Y, K, J, L of Sec. 3.2.2)
    Kern<k_Phi_hat3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, c->spec[F_PSI][nw], c->spec[F_PHI][nw], sp[1],
           c->Mdiag, sp[2]);
    ztrans(c, c->Wd, sp[2], dz[1]);   // dz[2..5] were taken at the start of the step
    Mom3 z{FLD(F_UZ, 0), FLD(F_UZ, -1), dz[0], dz[1], dz[2], dz[3], dz[4], dz[5], S[PFD_SRC_FZ],
           Lb[3], Lb[4], Lb[5], Lb[6]};
    Kern<k_mom_elem<true>>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, c->fld[F_PHI][nw], c->fld[F_PSI][nw], E2, c->Q2,
           FLD(F_UX, 0), FLD(F_UX, -1), FLD(F_UY, 0), FLD(F_UY, -1), FLD(F_P, 0), FLD(F_P, -1), S[PFD_SRC_FX],
           S[PFD_SRC_FY], Lb[0], Lb[1], Lb[2], z);
    // ---- P (eq. 77)
    Kern<k_P_rhs3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, Lb[0], Lb[3], S[PFD_SRC_WX], S[PFD_SRC_WY], ph[0],
           ph[1]);
    ztrans_n(c, 2, Wff, ph01, sp);
    Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_P, 0), sp[0], sp[1], 0, 1.0,
           (const double*)nullptr, 0.0, c->Mdiag, c->d_beta2, c->d_betad, c->srcS[PFD_SRC_F2],
           H(PFD_FAM_P, F_P, 0), H(PFD_FAM_P, F_P, -1), BB(PFD_FAM_P), c->r, c->spec[F_P][nw]);
    solve(c, PFD_FAM_P, BB(PFD_FAM_P), c->spec[F_P][nw], 1, 0, RR(PFD_FAM_P), !W(PFD_FAM_P));
    {
      const double* ins[2] = {c->spec[F_P][nw], c->spec[F_P][nw]};
      double* outs[2] = {c->fld[F_P][nw], dz[0]};
      ztrans_n(c, 2, Wid, ins, outs);
    }
    // ---- u (eq. 78)
    Kern<k_gradP_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, c->fld[F_P][nw], (const double*)dz[0], Lb[1], Lb[2],
           Lb[4]);
    Kern<k_u_rhs3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, Lb[1], Lb[5], Lb[2], Lb[6], Lb[4], c->bm_open,
           S[PFD_SRC_F1X], S[PFD_SRC_F1Y], S[PFD_SRC_F1Z], ph[0], ph[1], ph[2], ph[3], ph[4]);
    {
      const double* ins[5] = {ph[0], ph[1], ph[2], ph[3], ph[4]};
      ztrans_n(c, 5, Wff, ins, sp);
    }
    const int uf[3] = {F_UX, F_UY, F_UZ};
    const int ws[3] = {PFD_SRC_WX, PFD_SRC_WY, PFD_SRC_WZ};
    const double* Bs[3] = {sp[1], sp[3], nullptr};
    const double* As[3] = {sp[0], sp[2], sp[4]};
    for (int i = 0; i < 3; ++i)
      Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, LR(PFD_FAM_U, i), As[i], Bs[i], 0, 1.0,
             (const double*)nullptr, 0.0, c->Mdiag, c->d_beta2, c->d_betad, c->srcS[ws[i]],
             H(PFD_FAM_U, uf[i], 0), H(PFD_FAM_U, uf[i], -1), BB(PFD_FAM_U) + i * tot, c->r + i * tot,
             c->spec[uf[i]][nw]);
    solve(c, PFD_FAM_U, BB(PFD_FAM_U), c->spec[F_UX][nw], 3, 0, RR(PFD_FAM_U), !W(PFD_FAM_U));   // one stack
    {
      const double* ins[3] = {c->spec[F_UX][nw], c->spec[F_UY][nw], c->spec[F_UZ][nw]};
      double* outs[3] = {c->fld[F_UX][nw], c->fld[F_UY][nw], c->fld[F_UZ][nw]};
      ztrans_n(c, 3, Wfi, ins, outs);
    }
  }
  Kern<k_check_finite>::launch(c, PFD_PROF_OTHER, dim3(std::min(1024L, (long)nblk(tot))), dim3(WG), 0, st, tot,
         (const double*)c->fld[F_PHI][nw], equilibrium ? (const double*)nullptr : (const double*)c->fld[F_UX][nw],
         c->d_status);
  c->cur = nw;
  return hipGetLastError();
}

// one fixed-point iteration of Remark 3.1 in 3D (phi* = phi^n), physical Vin -> Vout
hipError_t potential_iteration_3d(pfd_ctx* c, const double* Vin, double* Vout) {
  Geo g = c->geo;
  Par P = c->par;
  P.cs_n = 1.0;
  P.cs_o = 0.0;
  dim3 eg(g.nx * g.ny, (c->planes + g.ppw - 1) / g.ppw), eb(((g.ppw * c->nq + 63) / 64) * 64);
  const long tot = (long)c->planes * c->Ng;
  const dim3 ng(nblk(tot)), nb(WG);
  hipStream_t st = c->stream;
  const bool warm = warm_start(c, PFD_FAM_V);
  double **ph = c->ph, **sp = c->sp, **dz = c->dz;
  refresh_spectral_sources(c);
  const double* phn = FLD(F_PHI, 0);
  ztrans(c, c->Dz, Vin, dz[0]);
  Kern<k_V_elem>::launch(c, PFD_PROF_ELEM, eg, eb, 0, st, g, P, phn, phn, Vin, Vin, c->Lb[0]);
  Kern<k_V_rhs3>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, c->Lb[0], c->Mdiag, c->src[PFD_SRC_FV], phn, phn, dz[0],
         ph[0], ph[1]);
  {
    const double* Wff[3] = {c->Wf, c->Wf, c->Wf};
    const double* ins[3] = {ph[0], ph[1], Vin};
    ztrans_n(c, warm ? 3 : 2, Wff, ins, sp);
  }
  double* Vh = c->spec[F_V][1 - c->cur];
  Kern<k_spec_rhs>::launch(c, PFD_PROF_NODAL, ng, nb, 0, st, g, P, c->lift[PFD_FAM_V], sp[0], sp[1], 0, 1.0 / P.eps0,
         (const double*)nullptr, 0.0, c->Mdiag, c->d_beta2, c->d_betad, c->srcS[PFD_SRC_VD],
         warm ? (const double*)sp[2] : nullptr, (const double*)sp[2], c->b[0], c->r, Vh);
  hipError_t e = solve(c, PFD_FAM_V, c->b[0], Vh, 1, 0, warm ? nullptr : c->r, !warm);
  ztrans(c, c->Wi, Vh, Vout);
  return e != hipSuccess ? e : hipGetLastError();
}

// spectral copy of a physical field: spec = Wf phys
hipError_t to_spectral(pfd_ctx* c, const double* phys, double* spec) {
  ztrans(c, c->Wf, phys, spec);
  return hipGetLastError();
}

}  // namespace pfd
