// One-time FP64 host set-up of the constant operators (remark after Algorithm 2:
// every coefficient matrix of the step is time-independent and is prepared once).
//
//  * GLL rule of order K: interior nodes are the eigenvalues of the Jacobi matrix
//    of the (1,1) Gauss-Jacobi polynomials (P_K' is proportional to P_{K-1}^{(1,1)}),
//    weights 2/(K(K+1) P_K(x)^2); Lagrange derivative matrix from barycentric
//    weights.
//  * 1D assembled stiffness and (diagonal, GLL-collocated) mass along x and y.
//    On a tensor-product mesh with collocated GLL quadrature the 2D operator
//    int grad u . grad v + c int u v is exactly  Kx (x) My + Mx (x) Ky + c Mx (x) My.
//  * Generalised eigen-decompositions Kd S = Md S Lambda, S^T Md S = I, per
//    direction and boundary-condition combination (fast diagonalisation,
//    Lynch, Rice & Thomas 1964), by cyclic Jacobi rotations.
#include "pfd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pfd {

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix A (row-major,
// destroyed).  On return lam holds the eigenvalues, V (row-major) the
// eigenvectors as columns, sorted by ascending eigenvalue.
void sym_eig(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = a(i, j) * a(i, j);
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        double app = a(p, p), aqq = a(q, q);
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // rows/cols p, q
          double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  lam.resize(n);
  std::vector<double> W((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    lam[j] = a(idx[j], idx[j]);
    for (int k = 0; k < n; ++k) W[(size_t)k * n + j] = V[(size_t)k * n + idx[j]];
  }
  V.swap(W);
}

static double legendre_val(int K, double x) {
  double p0 = 1.0, p1 = x;
  if (K == 0) return 1.0;
  for (int n = 1; n < K; ++n) {
    double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

void gll_rule(int K, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D) {
  const int n = K + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[K] = 1.0;
  if (K >= 2) {
    int m = K - 1;  // interior nodes: roots of P_{K-1}^{(1,1)}
    std::vector<double> J((size_t)m * m, 0.0), lam, V;
    for (int i = 1; i < m; ++i) {  // off-diagonal b_i = sqrt(i(i+2)/((2i+1)(2i+3)))
      double b = std::sqrt((double)i * (i + 2) / ((2.0 * i + 1) * (2.0 * i + 3)));
      J[(size_t)(i - 1) * m + i] = b;
      J[(size_t)i * m + (i - 1)] = b;
    }
    sym_eig(m, J, lam, V);
    for (int i = 0; i < m; ++i) x[i + 1] = lam[i];
    // symmetrise to remove rounding asymmetry of the eigen-solver
    for (int i = 0; i <= K / 2; ++i) {
      double s = 0.5 * (x[K - i] - x[i]);
      x[i] = -s;
      x[K - i] = s;
    }
    if (K % 2 == 0) x[K / 2] = 0.0;
  }
  for (int j = 0; j < n; ++j) {
    double p = legendre_val(K, x[j]);
    w[j] = 2.0 / (K * (K + 1.0) * p * p);
  }
  // barycentric weights bw_j = 1 / prod_{k != j} (x_j - x_k)
  std::vector<double> bw(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) bw[j] /= (x[j] - x[k]);
  D.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      double v = (bw[j] / bw[i]) / (x[i] - x[j]);
      D[(size_t)i * n + j] = v;
      diag -= v;
    }
    D[(size_t)i * n + i] = diag;
  }
}

// Assembled 1D stiffness (dense) and lumped mass along one direction.
void assemble_1d(int ne, const double* bp, int K, bool periodic, const std::vector<double>& w,
                 const std::vector<double>& D, std::vector<double>& Kd, std::vector<double>& Md,
                 std::vector<double>& coord, const std::vector<double>& xi) {
  int N = ne * K + 1 - (periodic ? 1 : 0);
  Kd.assign((size_t)N * N, 0.0);
  Md.assign(N, 0.0);
  coord.assign(N, 0.0);
  const int n = K + 1;
  for (int e = 0; e < ne; ++e) {
    double h = bp[e + 1] - bp[e];
    for (int a = 0; a < n; ++a) {
      const int gi = e * K + a;
      const bool wrap = periodic && gi == N;   // last node identified with node 0
      const int i = wrap ? 0 : gi;
      if (!wrap) coord[i] = bp[e] + 0.5 * h * (xi[a] + 1.0);
      Md[i] += 0.5 * h * w[a];
      for (int b = 0; b < n; ++b) {
        const int gj = e * K + b;
        const int j = (periodic && gj == N) ? 0 : gj;
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += w[q] * D[(size_t)q * n + a] * D[(size_t)q * n + b];
        Kd[(size_t)i * N + j] += 2.0 / h * s;
      }
    }
  }
}

// Fast-diagonalisation factors for one direction with Dirichlet flags at the
// two ends (ignored when periodic).  Dirichlet rows of S are zero.
// Refines an approximate orthonormal eigenbasis Q (m x m, column j an eigenvector, from the
// FP64 Jacobi above) of the symmetric B_ab = K1[fa][fb] / sqrt(M[fa] M[fb]) in extended
// precision (long double, 64-bit significand): two Newton-Schulz steps Q <- Q (3I - Q^T Q)/2
// restore orthonormality, C = Q^T B Q is then diagonal up to the FP64 Jacobi's residual, and
// cyclic Jacobi sweeps on C (a rotation where |c_pq| > u sqrt(c_pp c_qq), the relative
// criterion of Demmel & Veselic 1992, so small eigenvalues keep their relative accuracy) are
// accumulated into Q.  With the exact null vector w (singular operator: no Dirichlet node),
// column 0 is set to w, the others are projected off it, and the sweeps leave column 0 out.
// The FP64 Jacobi alone stops relative to the largest eigenvalues, which left the smooth
// (small-eigenvalue) eigenvectors, and so the fast-diagonalisation inverse, accurate to only
// about 1e-12 on a 161-node operator.
static void refine_eig_ld(int m, const std::vector<int>& fr, const std::vector<double>& K1,
                          const std::vector<double>& M1, int N, bool singular, std::vector<double>& lam,
                          std::vector<double>& Qd) {
  typedef long double LD;
  std::vector<LD> B((size_t)m * m), Q((size_t)m * m), T((size_t)m * m), G((size_t)m * m);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      B[(size_t)a * m + b] = (LD)K1[(size_t)fr[a] * N + fr[b]] / sqrtl((LD)M1[fr[a]] * (LD)M1[fr[b]]);
  for (size_t i = 0; i < Q.size(); ++i) Q[i] = Qd[i];
  auto matmul_tn = [&](const std::vector<LD>& X, const std::vector<LD>& Y, std::vector<LD>& Z) {   // Z = X^T Y
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        LD acc = 0.0L;
        for (int k = 0; k < m; ++k) acc += X[(size_t)k * m + i] * Y[(size_t)k * m + j];
        Z[(size_t)i * m + j] = acc;
      }
  };
  auto newton_schulz = [&]() {
    matmul_tn(Q, Q, G);   // G = Q^T Q
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) G[(size_t)i * m + j] = (i == j ? 1.5L : 0.0L) - 0.5L * G[(size_t)i * m + j];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        LD acc = 0.0L;
        for (int k = 0; k < m; ++k) acc += Q[(size_t)i * m + k] * G[(size_t)k * m + j];
        T[(size_t)i * m + j] = acc;
      }
    Q.swap(T);
  };
  int j0 = 0;
  if (singular) {
    std::vector<LD> wv(m);
    LD nrm = 0.0L;
    for (int a = 0; a < m; ++a) {
      wv[a] = sqrtl((LD)M1[fr[a]]);
      nrm += wv[a] * wv[a];
    }
    nrm = sqrtl(nrm);
    for (int a = 0; a < m; ++a) wv[a] /= nrm;
    // the FP64 Jacobi sorted the null pair first; replace it by w and project the rest off w
    for (int a = 0; a < m; ++a) Q[(size_t)a * m] = wv[a];
    for (int j = 1; j < m; ++j) {
      LD dot = 0.0L;
      for (int a = 0; a < m; ++a) dot += wv[a] * Q[(size_t)a * m + j];
      for (int a = 0; a < m; ++a) Q[(size_t)a * m + j] -= dot * wv[a];
    }
    j0 = 1;
  }
  newton_schulz();
  newton_schulz();
  // C = Q^T B Q
  std::vector<LD> BQ((size_t)m * m), C((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      LD acc = 0.0L;
      for (int k = 0; k < m; ++k) acc += B[(size_t)i * m + k] * Q[(size_t)k * m + j];
      BQ[(size_t)i * m + j] = acc;
    }
  matmul_tn(Q, BQ, C);
  auto c = [&](int i, int j) -> LD& { return C[(size_t)i * m + j]; };
  const LD u = 1.1e-19L;
  for (int sweep = 0; sweep < 12; ++sweep) {
    int rot = 0;
    for (int p = j0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const LD apq = c(p, q);
        if (fabsl(apq) <= u * sqrtl(fabsl(c(p, p) * c(q, q)))) continue;
        ++rot;
        const LD theta = (c(q, q) - c(p, p)) / (2.0L * apq);
        const LD t = (theta >= 0 ? 1.0L : -1.0L) / (fabsl(theta) + sqrtl(theta * theta + 1.0L));
        const LD cs = 1.0L / sqrtl(t * t + 1.0L), sn = t * cs;
        for (int k = 0; k < m; ++k) {
          const LD akp = c(k, p), akq = c(k, q);
          c(k, p) = cs * akp - sn * akq;
          c(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {
          const LD apk = c(p, k), aqk = c(q, k);
          c(p, k) = cs * apk - sn * aqk;
          c(q, k) = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const LD vkp = Q[(size_t)k * m + p], vkq = Q[(size_t)k * m + q];
          Q[(size_t)k * m + p] = cs * vkp - sn * vkq;
          Q[(size_t)k * m + q] = sn * vkp + cs * vkq;
        }
      }
    if (rot == 0) break;
  }
  // ascending eigenvalues (the null pair stays first)
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin() + j0, idx.end(), [&](int x, int y) { return c(x, x) < c(y, y); });
  lam.assign(m, 0.0);
  std::vector<double> W((size_t)m * m);
  for (int j = 0; j < m; ++j) {
    lam[j] = (singular && j == 0) ? 0.0 : (double)c(idx[j], idx[j]);
    for (int k = 0; k < m; ++k) W[(size_t)k * m + j] = (double)(Q[(size_t)k * m + idx[j]] / sqrtl((LD)M1[fr[k]]));
  }
  Qd.swap(W);   // now S restricted to the free nodes: Q / sqrt(M)
}

void build_dir1d(Dir1D& d, int ne, const double* bp, int K, bool periodic, bool dir_lo, bool dir_hi,
                 const std::vector<double>& xi, const std::vector<double>& w,
                 const std::vector<double>& D) {
  assemble_1d(ne, bp, K, periodic, w, D, d.K1, d.M1, d.coord, xi);
  const int N = (int)d.M1.size();
  d.N = N;
  d.periodic = periodic;
  d.dir.assign(N, 0);
  if (!periodic) {
    if (dir_lo) d.dir[0] = 1;
    if (dir_hi) d.dir[N - 1] = 1;
  }
  std::vector<int> fr;
  for (int i = 0; i < N; ++i)
    if (!d.dir[i]) fr.push_back(i);
  const int m = (int)fr.size();
  std::vector<double> B((size_t)m * m), lam, Q;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      B[(size_t)a * m + b] = d.K1[(size_t)fr[a] * N + fr[b]] /
                             std::sqrt(d.M1[fr[a]] * d.M1[fr[b]]);
  sym_eig(m, B, lam, Q);
  d.singular = (m == N);  // no Dirichlet node: constants are in the kernel
  refine_eig_ld(m, fr, d.K1, d.M1, N, d.singular, lam, Q);   // Q <- eigenvectors / sqrt(M)
  d.S.assign((size_t)N * N, 0.0);
  d.lam.assign(N, 1.0);
  for (int j = 0; j < m; ++j) {
    d.lam[j] = lam[j];
    for (int a = 0; a < m; ++a) d.S[(size_t)fr[a] * N + j] = Q[(size_t)a * m + j];
  }
  d.nfree = m;
  // banded, transposed copy of the stiffness for the residual kernel
  d.Kb.assign((size_t)(2 * K + 1) * N, 0.0);
  for (int i = 0; i < N; ++i) {
    const int dhi = (periodic && N == 2 * K) ? K - 1 : K;  // two periodic elements: -K and +K coincide
    for (int dd = -K; dd <= dhi; ++dd) {
      int j = i + dd;
      if (periodic) j = (j + N) % N;
      else if (j < 0 || j >= N) continue;
      d.Kb[(size_t)(dd + K) * N + i] = d.K1[(size_t)i * N + j];
    }
  }
}

}  // namespace pfd

namespace pfd {

// Gap-node Schur complement of the potential operator with partial electrode sets.
// The fast-diagonalisation base operator A_D treats the whole bottom row as Dirichlet; the
// true operator releases the gap nodes G of that row (bottom nodes outside the electrode
// segments).  With F the free nodes of A_D:
//   S_G = A_GG - A_GF A_FF^{-1} A_FG,
// where A_FG couples a gap node (g, 0) only to (g, iy), iy = 1..K, through Mx[g] Ky[iy][0],
// and A_GG = My[0] Kx[g_i][g_j] + delta_ij Mx[g_i] (Ky[0][0] + c My[0]).
// Returns S_G^{-1} (row-major n_g x n_g) for the total shift c.
void electrode_schur_inverse(const Dir1D& dx, const Dir1D& dy, const std::vector<int>& gap, int K, double c,
                             std::vector<double>& Sinv) {
  const int Nx = dx.N, Ny = dy.N, ng = (int)gap.size();
  const int kmax = std::min(K, Ny - 1);
  std::vector<double> S((size_t)ng * ng, 0.0);
  std::vector<double> u(Ny), T((size_t)Ny * Nx);
  for (int j = 0; j < ng; ++j) {
    const int gj = gap[j];
    // z = A_FG e_j: column gj, rows 1..K, value Mx[gj] Ky[iy][0]
    // w = A_FF^{-1} z = Sy [ (Sy^T z Sx) ./ (ly + lx + c) ] Sx^T ; z has one column
    for (int a = 0; a < Ny; ++a) {
      double acc = 0.0;
      for (int iy = 1; iy <= kmax; ++iy) acc += dy.S[(size_t)iy * Ny + a] * dx.M1[gj] * dy.K1[(size_t)iy * Ny];
      u[a] = acc;
    }
    for (int a = 0; a < Ny; ++a)
      for (int b = 0; b < Nx; ++b) {
        const double den = dy.lam[a] + dx.lam[b] + c;
        T[(size_t)a * Nx + b] = den != 0.0 ? u[a] * dx.S[(size_t)gj * Nx + b] / den : 0.0;
      }
    for (int i = 0; i < ng; ++i) {
      const int gi = gap[i];
      // (A_GF w)_i = Mx[gi] sum_{iy=1..K} Ky[0][iy] w(gi, iy),  w(gi, iy) = sum_a Sy[iy][a] ta[a]
      for (int a = 0; a < Ny; ++a) {
        double acc = 0.0;
        for (int b = 0; b < Nx; ++b) acc += T[(size_t)a * Nx + b] * dx.S[(size_t)gi * Nx + b];
        u[a] = acc;  // (reuses u as ta: u of column j is no longer needed)
      }
      double agw = 0.0;
      for (int iy = 1; iy <= kmax; ++iy) {
        double w = 0.0;
        for (int a = 0; a < Ny; ++a) w += dy.S[(size_t)iy * Ny + a] * u[a];
        agw += dy.K1[(size_t)iy] * w;
      }
      agw *= dx.M1[gi];
      double agg = dy.M1[0] * dx.K1[(size_t)gi * Nx + gj];
      if (i == j) agg += dx.M1[gi] * (dy.K1[0] + c * dy.M1[0]);
      S[(size_t)i * ng + j] = agg - agw;
    }
  }
  // Gauss-Jordan inverse with partial pivoting (S is symmetric positive definite)
  Sinv.assign((size_t)ng * ng, 0.0);
  for (int i = 0; i < ng; ++i) Sinv[(size_t)i * ng + i] = 1.0;
  for (int col = 0; col < ng; ++col) {
    int piv = col;
    for (int r = col + 1; r < ng; ++r)
      if (std::fabs(S[(size_t)r * ng + col]) > std::fabs(S[(size_t)piv * ng + col])) piv = r;
    if (piv != col)
      for (int k = 0; k < ng; ++k) {
        std::swap(S[(size_t)col * ng + k], S[(size_t)piv * ng + k]);
        std::swap(Sinv[(size_t)col * ng + k], Sinv[(size_t)piv * ng + k]);
      }
    const double d = S[(size_t)col * ng + col];
    for (int k = 0; k < ng; ++k) {
      S[(size_t)col * ng + k] /= d;
      Sinv[(size_t)col * ng + k] /= d;
    }
    for (int r = 0; r < ng; ++r) {
      if (r == col) continue;
      const double f = S[(size_t)r * ng + col];
      if (f == 0.0) continue;
      for (int k = 0; k < ng; ++k) {
        S[(size_t)r * ng + k] -= f * S[(size_t)col * ng + k];
        Sinv[(size_t)r * ng + k] -= f * Sinv[(size_t)col * ng + k];
      }
    }
  }
}

}  // namespace pfd
