// C-ABI of the pfd library: context set-up, field I/O and the stepping entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>

#include "pfd_internal.h"

using namespace pfd;

static std::string g_create_err;

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      c->err = std::string("HIP error: ") + hipGetErrorString(_e) + " at " #expr; \
      return PFD_EHIP;                                                            \
    }                                                                             \
  } while (0)

extern "C" const char* pfd_status_string(pfd_status s) {
  switch (s) {
    case PFD_OK: return "PFD_OK";
    case PFD_EINVAL: return "PFD_EINVAL";
    case PFD_ENOMEM: return "PFD_ENOMEM";
    case PFD_EHIP: return "PFD_EHIP";
    case PFD_ENONFINITE: return "PFD_ENONFINITE";
    case PFD_ENOCONV: return "PFD_ENOCONV";
    case PFD_ESTATE: return "PFD_ESTATE";
    case PFD_ENOTIMPL: return "PFD_ENOTIMPL";
  }
  return "PFD_UNKNOWN";
}

extern "C" const char* pfd_last_error(const pfd_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

namespace {

struct Layout {
  int Nx, Ny, planes, is3d;
  long Ng, Nl;
  size_t bytes;
};

// work-groups of the largest residual launch (three stacked components, either residual kernel)
long refine_blocks(int Ny, int planes, long Pg) {
  return std::max(3 * Pg / 256 + 1, (long)((Ny + 15) / 16) * 3 * planes) + 16;
}

pfd_status validate(const pfd_problem* p, Layout* L, std::string* err) {
  if (!p) { *err = "null problem"; return PFD_EINVAL; }
  const pfd_mesh& m = p->mesh;
  // the (K+1)^2 nodes of an element are one work-group of at most 256 threads
  if (m.K < 2 || m.K > PFD_KMAX_STEP) { *err = "K must be in [2,15]"; return PFD_EINVAL; }
  if (m.nx < 1 || m.ny < 1 || !m.xb || !m.yb) { *err = "bad element counts or breakpoints"; return PFD_EINVAL; }
  if (m.periodic_x && m.nx < 2) { *err = "periodic x needs nx >= 2"; return PFD_EINVAL; }
  for (int i = 0; i < m.nx; ++i)
    if (!(m.xb[i + 1] > m.xb[i])) { *err = "x breakpoints must increase"; return PFD_EINVAL; }
  for (int i = 0; i < m.ny; ++i)
    if (!(m.yb[i + 1] > m.yb[i])) { *err = "y breakpoints must increase"; return PFD_EINVAL; }
  const pfd_params& q = p->par;
  if (!(q.dt > 0) || !(q.eta > 0) || !(q.lambda > 0) || !(q.gamma1 > 0)) {
    *err = "dt, eta, lambda, gamma1 must be positive"; return PFD_EINVAL;
  }
  if (!(q.rho1 > 0) || !(q.rho2 > 0) || !(q.mu1 > 0) || !(q.mu2 > 0) || !(q.eps1 > 0) || !(q.eps2 > 0)) {
    *err = "material properties must be positive"; return PFD_EINVAL;
  }
  if (q.bdf_order != 1 && q.bdf_order != 2) { *err = "bdf_order must be 1 or 2"; return PFD_EINVAL; }
  if (p->precision == PFD_REFINED_BF16) {
    *err = "BF16 corrections are not built (measured to need more corrections than they save)";
    return PFD_ENOTIMPL;
  }
  if (p->precision != PFD_PLAIN_FP64 && p->precision != PFD_REFINED_FP32) { *err = "bad precision"; return PFD_EINVAL; }
  if (p->refine_max < 0 || p->refine_max > 64 || !(p->refine_tol >= 0.0) || !(p->refine_tol < 1.0)) {
    *err = "refine_max must be in [0,64] and refine_tol in [0,1)"; return PFD_EINVAL;
  }
  if (m.nz < 0 || m.nz == 1 || (m.nz > 0 && m.nz % 2)) { *err = "nz must be 0 (2D) or even >= 2"; return PFD_EINVAL; }
  if (m.nz > 0 && !(m.lz > 0)) { *err = "lz must be positive in 3D"; return PFD_EINVAL; }
  if (m.nz > 512) { *err = "nz above 512 is not supported"; return PFD_EINVAL; }
  if (m.nbatch < 1 || (m.nz > 0 && m.nbatch != 1)) { *err = "nbatch must be >= 1 (and 1 in 3D)"; return PFD_EINVAL; }
  if (p->bc.n_electrodes < 0 || (p->bc.n_electrodes > 0 && (!p->bc.electrode_x0 || !p->bc.electrode_x1))) {
    *err = "bad electrode list"; return PFD_EINVAL;
  }
  for (int i = 0; i < p->bc.n_electrodes; ++i) {
    // segment ends must lie on element edges
    const double e0 = p->bc.electrode_x0[i], e1 = p->bc.electrode_x1[i];
    bool ok0 = false, ok1 = false;
    const double tol = 1e-10 * (m.xb[m.nx] - m.xb[0]);
    for (int k = 0; k <= m.nx; ++k) {
      if (std::fabs(m.xb[k] - e0) <= tol) ok0 = true;
      if (std::fabs(m.xb[k] - e1) <= tol) ok1 = true;
    }
    if (!ok0 || !ok1 || !(e1 > e0)) { *err = "electrode segments must span element edges"; return PFD_EINVAL; }
  }
  for (int s = 0; s < 4; ++s) {
    if (m.periodic_x && s >= PFD_LEFT) continue;
    if (p->bc.side_type[s] != PFD_WALL && p->bc.side_type[s] != PFD_OPEN) { *err = "side type must be WALL or OPEN"; return PFD_EINVAL; }
  }
  bool anyV = p->bc.n_electrodes > 0;
  for (int s = 0; s < 4; ++s)
    if (p->bc.pot_dirichlet[s] && !(m.periodic_x && s >= PFD_LEFT)) anyV = true;
  if (!anyV) { *err = "the potential needs a Dirichlet side"; return PFD_EINVAL; }
  L->Nx = m.nx * m.K + 1 - (m.periodic_x ? 1 : 0);
  L->Ny = m.ny * m.K + 1;
  if (L->Nx > PFD_NMAX || L->Ny > PFD_NMAX) { *err = "more than 320 nodes along a direction"; return PFD_EINVAL; }
  L->is3d = m.nz > 0;
  L->planes = L->is3d ? m.nz : m.nbatch;
  L->Ng = (long)L->Nx * L->Ny;
  L->Nl = (long)m.nx * m.ny * (m.K + 1) * (m.K + 1);
  const long Pg = L->planes * L->Ng, Pl = L->planes * L->Nl;
  size_t dbl = 0;
  dbl += (size_t)F_NSTATE * 2 * Pg;      // state
  dbl += (size_t)PFD_NSRC * Pg;          // sources
  dbl += (L->is3d ? 7 : 3) * (size_t)Pl; // element-local buffers
  if (L->is3d) {
    dbl += 14 * (size_t)Pg;              // spectral state
    dbl += 16 * (size_t)Pg;              // physical / spectral / z-derivative temporaries
    dbl += 5 * (size_t)Pg;               // spectral Dirichlet data
    dbl += 4 * (size_t)m.nz * m.nz + 64; // DFT matrices
    dbl += (size_t)m.nz + 2 + 64;        // FFT twiddles
  }
  dbl += 3 * (size_t)Pg;                 // right sides
  dbl += 13 * (size_t)Pg;                // r (3), U, Q2, tmp (3), tmp2 (3), zero, Ybuf
  dbl += 14 * (size_t)Pg;                // right sides per family and level (u: three components)
  dbl += 15 * (size_t)L->planes + 64;    // family shifts, repeated per stacked component
  dbl += (size_t)L->planes * PFD_STAT_NB * 8;  // diagnostics partials
  if (p->bc.n_electrodes > 0) dbl += (size_t)L->planes * (L->Nx * (size_t)L->Nx + L->Nx) + 4 * (size_t)L->Nx;
  dbl += 7 * (size_t)L->Ng;              // boundary masses, mass
  const int NN = std::max(L->Nx, L->Ny);
  dbl += 8 * (3 * (size_t)NN * NN + 3 * NN + 8);  // up to 8 distinct 1D operators
  dbl += 8 * (size_t)NN * NN;            // float copies (as doubles, generous)
  const size_t NP = (size_t)((NN + 15) & ~15);
  dbl += 8 * 3 * NP * NP + 64;           // S, S^T in fragment order, double and float
  dbl += 2 * (size_t)(m.nx + m.ny + 2) + (PFD_KMAX + 1) * (PFD_KMAX + 2);
  dbl += 48 * (size_t)L->planes + 1280;  // shifts, norms, reductions (1024 block maxima)
  dbl += 2 * (size_t)refine_blocks(L->Ny, L->planes, Pg) + 5 * (size_t)L->planes + 64;  // refinement test
  L->bytes = dbl * sizeof(double) + 256 * 1024;  // alignment slack (256 B per allocation)
  return PFD_OK;
}

void* carve(pfd_ctx* c, size_t bytes) {
  size_t off = (c->ws_used + 255) & ~(size_t)255;
  if (off + bytes > c->ws_bytes) {
    c->ws_fail = true;
    return nullptr;
  }
  c->ws_used = off + bytes;
  return c->ws + off;
}

}  // namespace

extern "C" pfd_status pfd_workspace_query(const pfd_problem* prob, size_t* dev_bytes) {
  Layout L;
  pfd_status s = validate(prob, &L, &g_create_err);
  if (s != PFD_OK) return s;
  if (dev_bytes) *dev_bytes = L.bytes;
  return PFD_OK;
}

extern "C" pfd_status pfd_create(const pfd_problem* prob, void* dev_ws, size_t dev_bytes, void* stream,
                                 pfd_ctx** out) {
  if (!out) { g_create_err = "null output pointer"; return PFD_EINVAL; }
  *out = nullptr;
  Layout L;
  pfd_status st = validate(prob, &L, &g_create_err);
  if (st != PFD_OK) return st;
  if (!dev_ws || dev_bytes < L.bytes) { g_create_err = "workspace too small"; return PFD_ENOMEM; }
  if (((uintptr_t)dev_ws) & 255) { g_create_err = "workspace must be 256-byte aligned"; return PFD_EINVAL; }
  pfd_ctx* c = new pfd_ctx();
  c->prob = *prob;
  c->prob.mesh.xb = nullptr;  // host pointers are not kept
  c->prob.mesh.yb = nullptr;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  c->ws = (char*)dev_ws;
  c->ws_bytes = dev_bytes;
  c->Nx = L.Nx; c->Ny = L.Ny; c->planes = L.planes; c->is3d = L.is3d;
  c->Ng = L.Ng; c->Nl = L.Nl;
  const pfd_mesh& m = prob->mesh;
  const int K = m.K;
  c->K = K; c->n = K + 1; c->nq = (K + 1) * (K + 1);
  gll_rule(K, c->xi, c->w, c->D);

  // ---- derived constants (Sec. 3.1, eq. 44)
  const pfd_params& q = prob->par;
  Par& P = c->par;
  P.rho1 = q.rho1; P.rho2 = q.rho2; P.mu1 = q.mu1; P.mu2 = q.mu2; P.eps1 = q.eps1; P.eps2 = q.eps2;
  P.lam = q.lambda; P.eta = q.eta; P.gamma1 = q.gamma1; P.dt = q.dt;
  P.gamma0 = (q.bdf_order == 2) ? 1.5 : 1.0;
  const double lg = q.lambda * q.gamma1;
  const double Slow = q.eta * q.eta * std::sqrt(4.0 * P.gamma0 / (lg * q.dt));
  P.S = q.S > 0 ? q.S : Slow;
  double rad = 1.0 - 4.0 * P.gamma0 / (lg * q.dt) * std::pow(q.eta, 4) / (P.S * P.S);
  if (rad < 0.0) rad = 0.0;
  P.alpha = -P.S / (2.0 * q.eta * q.eta) * (1.0 + std::sqrt(rad));
  P.c_psi = P.alpha + P.S / (q.eta * q.eta);
  P.c_phi = -P.alpha;
  P.eps0 = std::max(q.eps1, q.eps2);
  P.rho0 = std::min(q.rho1, q.rho2);
  P.nu_m = q.nu_m > 0 ? q.nu_m : std::max(q.mu1, q.mu2) / std::min(q.rho1, q.rho2);
  P.c_u = P.gamma0 / (P.nu_m * q.dt);
  P.cos_theta = std::cos(q.theta_s_deg * M_PI / 180.0);
  if (q.bdf_order == 2) { P.cs_n = 2.0; P.cs_o = -1.0; P.ch_n = 2.0; P.ch_o = -0.5; }
  else { P.cs_n = 1.0; P.cs_o = 0.0; P.ch_n = 1.0; P.ch_o = 0.0; }

  // ---- 1D operators per family and direction (deduplicated)
  const pfd_bcs& bc = prob->bc;
  const bool per = m.periodic_x != 0;
  auto side_dir = [&](int fam, int s) -> bool {
    if (per && s >= PFD_LEFT) return false;
    switch (fam) {
      case PFD_FAM_V: return bc.pot_dirichlet[s] != 0 || (s == PFD_BOTTOM && bc.n_electrodes > 0);
      case PFD_FAM_P: return bc.side_type[s] == PFD_OPEN;
      case PFD_FAM_U: return bc.side_type[s] == PFD_WALL;
      default: return false;
    }
  };
  std::map<std::tuple<int, int, int>, int> xkey, ykey;
  for (int f = 0; f < 5; ++f) {
    auto kx = std::make_tuple(per ? 2 : 0, (int)side_dir(f, PFD_LEFT), (int)side_dir(f, PFD_RIGHT));
    auto ky = std::make_tuple(0, (int)side_dir(f, PFD_BOTTOM), (int)side_dir(f, PFD_TOP));
    if (!xkey.count(kx)) {
      Dir1D d;
      build_dir1d(d, m.nx, m.xb, K, per, std::get<1>(kx), std::get<2>(kx), c->xi, c->w, c->D);
      xkey[kx] = (int)c->dirs.size();
      c->dirs.push_back(std::move(d));
    }
    if (!ykey.count(ky)) {
      Dir1D d;
      build_dir1d(d, m.ny, m.yb, K, false, std::get<1>(ky), std::get<2>(ky), c->xi, c->w, c->D);
      ykey[ky] = (int)c->dirs.size();
      c->dirs.push_back(std::move(d));
    }
    c->fam[f].ix = xkey[kx];
    c->fam[f].iy = ykey[ky];
  }
  const double shifts[5] = {0.0, P.c_psi, P.c_phi, 0.0, P.c_u};
  c->beta2.assign(c->planes, 0.0);
  c->betad.assign(c->planes, 0.0);
  std::vector<double> Wf, Wi, Wd, Dz;
  if (c->is3d) {
    // packed spectral planes: 0 = k 0, 1 = Nyquist, 2k / 2k+1 = Re / Im of mode k
    const int Nz = m.nz;
    const double Lz = m.lz;
    auto kof = [&](int p) { return p == 0 ? 0 : (p == 1 ? Nz / 2 : p / 2); };
    for (int p = 0; p < Nz; ++p) {
      const double beta = 2.0 * M_PI * kof(p) / Lz;
      c->beta2[p] = beta * beta;
      c->betad[p] = (p < 2) ? 0.0 : beta;   // Nyquist first derivative is 0 (reading R-nyq)
    }
    Wf.assign((size_t)Nz * Nz, 0.0); Wi = Wf; Wd = Wf; Dz = Wf;
    for (int j = 0; j < Nz; ++j) {
      const double sgn = (j % 2) ? -1.0 : 1.0;
      Wf[(size_t)0 * Nz + j] = 1.0 / Nz;
      Wf[(size_t)1 * Nz + j] = sgn / Nz;
      Wi[(size_t)j * Nz + 0] = 1.0;
      Wi[(size_t)j * Nz + 1] = sgn;
      for (int k = 1; k < Nz / 2; ++k) {
        const double th = 2.0 * M_PI * (double)((long)j * k % Nz) / Nz;
        const double cs = std::cos(th), sn = std::sin(th), beta = 2.0 * M_PI * k / Lz;
        Wf[(size_t)(2 * k) * Nz + j] = cs / Nz;
        Wf[(size_t)(2 * k + 1) * Nz + j] = -sn / Nz;
        Wi[(size_t)j * Nz + 2 * k] = 2.0 * cs;
        Wi[(size_t)j * Nz + 2 * k + 1] = -2.0 * sn;
        Wd[(size_t)j * Nz + 2 * k] = -2.0 * beta * sn;
        Wd[(size_t)j * Nz + 2 * k + 1] = -2.0 * beta * cs;
      }
    }
    for (int i = 0; i < Nz; ++i)
      for (int j = 0; j < Nz; ++j) {
        double acc = 0.0;
        for (int p = 0; p < Nz; ++p) acc += Wd[(size_t)i * Nz + p] * Wf[(size_t)p * Nz + j];
        Dz[(size_t)i * Nz + j] = acc;
      }
  }

  // ---- carve the workspace
  const long Pg = (long)c->planes * c->Ng, Pl = (long)c->planes * c->Nl;
  auto D = [&](long n) { return (double*)carve(c, sizeof(double) * n); };
  // the velocity components of a level are contiguous: their solves run as one plane stack
  for (int l = 0; l < 2; ++l) {
    double* blk = D(3 * Pg);
    c->fld[F_UX][l] = blk;
    c->fld[F_UY][l] = blk ? blk + Pg : nullptr;
    c->fld[F_UZ][l] = blk ? blk + 2 * Pg : nullptr;
  }
  for (int f = 0; f < F_NSTATE; ++f)
    if (f != F_UX && f != F_UY && f != F_UZ)
      for (int l = 0; l < 2; ++l) c->fld[f][l] = D(Pg);
  for (int s = 0; s < PFD_NSRC; ++s) c->src[s] = D(Pg);
  for (int i = 0; i < (c->is3d ? 7 : 3); ++i) c->Lb[i] = D(Pl);
  if (c->is3d) {
    for (int l = 0; l < 2; ++l) {
      double* blk = D(3 * Pg);
      c->spec[F_UX][l] = blk;
      c->spec[F_UY][l] = blk ? blk + Pg : nullptr;
      c->spec[F_UZ][l] = blk ? blk + 2 * Pg : nullptr;
    }
    for (int f : {F_P, F_PHI, F_PSI, F_V})
      for (int l = 0; l < 2; ++l) c->spec[f][l] = D(Pg);
    for (int i = 0; i < 5; ++i) c->ph[i] = D(Pg);
    for (int i = 0; i < 5; ++i) c->sp[i] = D(Pg);
    for (int i = 0; i < 6; ++i) c->dz[i] = D(Pg);
    for (int s : {PFD_SRC_VD, PFD_SRC_F2, PFD_SRC_WX, PFD_SRC_WY, PFD_SRC_WZ}) c->srcS[s] = D(Pg);
    const long NZ2 = (long)m.nz * m.nz;
    c->Wf = D(NZ2); c->Wi = D(NZ2); c->Wd = D(NZ2); c->Dz = D(NZ2);
    c->twr = D(m.nz / 2 + 1); c->twi = D(m.nz / 2 + 1);
  }
  {
    double* blk = D(3 * Pg);   // right sides, contiguous (stacked velocity components)
    for (int i = 0; i < 3; ++i) c->b[i] = blk ? blk + i * Pg : nullptr;
  }
  c->r = D(3 * Pg); c->U = D(Pg); c->Q2 = D(Pg); c->tmp = D(3 * Pg); c->tmp2 = D(3 * Pg);
  for (int f = 0; f < 5; ++f)
    for (int l = 0; l < 2; ++l) c->bh[f][l] = D((f == PFD_FAM_U ? 3 : 1) * Pg);
  double* zero = D(Pg);
  c->Ybuf = D(Pg);
  for (int s = 0; s < 4; ++s) c->bm_side[s] = D(c->Ng);
  c->bm_open = D(c->Ng); c->bm_wall = D(c->Ng); c->Mdiag = D(c->Ng);
  c->d_hx = D(m.nx); c->d_hy = D(m.ny);
  c->d_w = D(K + 1); c->d_D = D((long)(K + 1) * (K + 1));
  c->d_status = (int*)carve(c, 64);
  c->d_red = D(2 * 512);
  c->rpart_max = refine_blocks(c->Ny, c->planes, Pg);
  c->d_rpart = D(2 * c->rpart_max);
  c->d_gate = (int*)carve(c, 64);
  c->d_rstat = D(20);
  for (int f = 0; f < 5; ++f) c->d_anorm[f] = D(c->planes);
  c->d_stats = D((long)c->planes * PFD_STAT_NB * 8);
  c->d_part = D(32 * (long)c->planes);
  c->d_beta2 = D(c->planes); c->d_betad = D(c->planes);
  for (int f = 0; f < 5; ++f) c->fam[f].dshift = D(3 * c->planes);   // repeated per stacked component
  for (auto& d : c->dirs) {
    const long NN = (long)d.N * d.N;
    d.dS = D(NN); d.dST = D(NN); d.dKb = D((long)(2 * K + 1) * d.N); d.dlam = D(d.N); d.dM1 = D(d.N);
    d.dK0 = D(d.N); d.dKN = D(d.N);
    d.fS = (float*)carve(c, sizeof(float) * NN);
    d.fST = (float*)carve(c, sizeof(float) * NN);
    const long NP2 = (long)((d.N + 15) & ~15) * ((d.N + 15) & ~15);
    d.dSw = D(NP2); d.dSTw = D(NP2);
    d.fSw = (float*)carve(c, sizeof(float) * NP2);
    d.fSTw = (float*)carve(c, sizeof(float) * NP2);
    d.ddir = (unsigned char*)carve(c, d.N);
  }
  bool ok = !c->ws_fail && c->fld[0][0] && zero && c->fam[4].dshift && c->bh[PFD_FAM_U][1] && c->d_anorm[4];
  for (auto& d : c->dirs) ok = ok && d.ddir;
  if (!ok) { g_create_err = "workspace too small (layout)"; delete c; return PFD_ENOMEM; }
  (void)zero;

  // ---- host tables -> device (synchronous copies: set-up only)
  hipError_t e = hipStreamSynchronize(c->stream);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  for (auto& d : c->dirs) {
    if (e) break;
    const int N = d.N;
    std::vector<double> ST((size_t)N * N);
    std::vector<float> f1((size_t)N * N), f2((size_t)N * N);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        ST[(size_t)j * N + i] = d.S[(size_t)i * N + j];
        f1[(size_t)i * N + j] = (float)d.S[(size_t)i * N + j];
        f2[(size_t)j * N + i] = (float)d.S[(size_t)i * N + j];
      }
    std::vector<unsigned char> dd(N);
    for (int i = 0; i < N; ++i) dd[i] = d.dir[i] ? 1 : 0;
    e = up(d.dS, d.S.data(), 8 * N * N); if (e) break;
    e = up(d.dST, ST.data(), 8 * N * N); if (e) break;
    e = up(d.dKb, d.Kb.data(), 8 * (2 * K + 1) * N); if (e) break;
    e = up(d.dlam, d.lam.data(), 8 * N); if (e) break;
    e = up(d.dM1, d.M1.data(), 8 * N); if (e) break;
    e = up(d.fS, f1.data(), 4 * N * N); if (e) break;
    e = up(d.fST, f2.data(), 4 * N * N); if (e) break;
    {
      // MFMA fragment order of S and S^T as left operands: tile (mt, sl), lane, then the four
      // contraction entries k = 16 sl + 4 (lane / 16) + s of row 16 mt + lane % 16
      const int KS = (N + 15) / 16;
      const size_t NP2 = (size_t)KS * 16 * KS * 16;
      std::vector<double> w1(NP2, 0.0), w2(NP2, 0.0);
      std::vector<float> v1(NP2, 0.0f), v2(NP2, 0.0f);
      for (int mt = 0; mt < KS; ++mt)
        for (int sl = 0; sl < KS; ++sl)
          for (int lane = 0; lane < 64; ++lane)
            for (int q = 0; q < 4; ++q) {
              const int i = 16 * mt + (lane & 15), k = 16 * sl + 4 * (lane >> 4) + q;
              const size_t o = (((size_t)mt * KS + sl) * 64 + lane) * 4 + q;
              if (i < N && k < N) {
                w1[o] = d.S[(size_t)i * N + k];
                w2[o] = d.S[(size_t)k * N + i];
                v1[o] = (float)w1[o];
                v2[o] = (float)w2[o];
              }
            }
      e = up(d.dSw, w1.data(), 8 * NP2); if (e) break;
      e = up(d.dSTw, w2.data(), 8 * NP2); if (e) break;
      e = up(d.fSw, v1.data(), 4 * NP2); if (e) break;
      e = up(d.fSTw, v2.data(), 4 * NP2); if (e) break;
    }
    e = up(d.ddir, dd.data(), N); if (e) break;
    std::vector<double> k0(N), kn(N);
    for (int i = 0; i < N; ++i) {
      k0[i] = d.K1[(size_t)i * N];
      kn[i] = d.K1[(size_t)i * N + N - 1];
    }
    e = up(d.dK0, k0.data(), 8 * N); if (e) break;
    e = up(d.dKN, kn.data(), 8 * N); if (e) break;
  }
  // boundary and volume masses from the x/y 1D masses (any family's dirs share M1)
  const Dir1D& DX = c->dirs[c->fam[0].ix];
  const Dir1D& DY = c->dirs[c->fam[0].iy];
  std::vector<double> Md(c->Ng), bs[4], bo(c->Ng, 0.0), bw(c->Ng, 0.0);
  for (int s = 0; s < 4; ++s) bs[s].assign(c->Ng, 0.0);
  c->Mtot = 0.0;
  for (int iy = 0; iy < c->Ny; ++iy)
    for (int ix = 0; ix < c->Nx; ++ix) {
      Md[(long)iy * c->Nx + ix] = DX.M1[ix] * DY.M1[iy];
      c->Mtot += DX.M1[ix] * DY.M1[iy];
    }
  for (int ix = 0; ix < c->Nx; ++ix) {
    bs[PFD_BOTTOM][ix] = DX.M1[ix];
    bs[PFD_TOP][(long)(c->Ny - 1) * c->Nx + ix] = DX.M1[ix];
  }
  if (!per)
    for (int iy = 0; iy < c->Ny; ++iy) {
      bs[PFD_LEFT][(long)iy * c->Nx] = DY.M1[iy];
      bs[PFD_RIGHT][(long)iy * c->Nx + c->Nx - 1] = DY.M1[iy];
    }
  for (int s = 0; s < 4; ++s) {
    if (per && s >= PFD_LEFT) continue;
    for (long i = 0; i < c->Ng; ++i) {
      if (bc.side_type[s] == PFD_OPEN) bo[i] += bs[s][i];
      else bw[i] += bs[s][i];
    }
  }
  std::vector<double> hx(m.nx), hy(m.ny);
  for (int i = 0; i < m.nx; ++i) hx[i] = m.xb[i + 1] - m.xb[i];
  for (int i = 0; i < m.ny; ++i) hy[i] = m.yb[i + 1] - m.yb[i];
  std::vector<double> shp[5];
  for (int f = 0; f < 5; ++f) {
    Family& F = c->fam[f];
    F.shift = shifts[f];
    F.hshift.assign(c->planes, 0.0);
    bool sing = c->dirs[F.ix].singular && c->dirs[F.iy].singular;
    F.any_singular = false;
    for (int p = 0; p < c->planes; ++p) {
      F.hshift[p] = F.shift + c->beta2[p];
      if (sing && F.hshift[p] == 0.0) F.any_singular = true;
    }
  }
  // precision ladder and the refinement test's operator norms.  Per plane, the generalised
  // eigenvalues of (A, M) are lx_i + ly_j + c_p, so kappa = (max lx + max ly + c_p) /
  // (min lx + min ly + c_p) is the condition number of M^{-1/2} A M^{-1/2}, and ||A_p||_2 <=
  // max(M) (max lx + max ly + c_p).  An FP32 correction reduces the error by about kappa u32
  // (u32 = 2^-24), so planes with kappa u32 > 1/2 -- the singular ones (kappa infinite) in
  // particular -- take one FP64 correction instead (they must form a prefix of the planes,
  // which holds here: only the first Fourier plane can be singular).
  const double u32 = std::ldexp(1.0, -24);
  std::vector<double> an[5];
  for (int f = 0; f < 5; ++f) {
    const Dir1D& dx = c->dirs[c->fam[f].ix];
    const Dir1D& dy = c->dirs[c->fam[f].iy];
    auto mm = [](const Dir1D& d, double& lo, double& hi, double& mx) {
      lo = 1e300; hi = -1e300; mx = 0.0;
      for (int j = 0; j < d.nfree; ++j) { lo = std::min(lo, d.lam[j]); hi = std::max(hi, d.lam[j]); }
      for (int i = 0; i < d.N; ++i) mx = std::max(mx, d.M1[i]);
    };
    double xlo, xhi, xm, ylo, yhi, ym;
    mm(dx, xlo, xhi, xm);
    mm(dy, ylo, yhi, ym);
    an[f].assign(c->planes, 0.0);
    c->kappa_min[f] = 1e300;
    c->kappa_max[f] = 0.0;
    std::vector<char> need64(c->planes, 0);
    for (int p = 0; p < c->planes; ++p) {
      const double sh = c->fam[f].hshift[p];
      const double hi = xhi + yhi + sh, lo = xlo + ylo + sh;
      an[f][p] = xm * ym * hi;
      const double kap = lo > 1e-12 * hi ? hi / lo : HUGE_VAL;
      c->kappa_min[f] = std::min(c->kappa_min[f], kap);
      c->kappa_max[f] = std::max(c->kappa_max[f], kap);
      need64[p] = kap * u32 > 0.5;
    }
    int n64 = 0;
    while (n64 < c->planes && need64[n64]) ++n64;
    for (int p = n64; p < c->planes; ++p)
      if (need64[p]) n64 = c->planes;   // not a prefix: the whole family in FP64
    if (f == PFD_FAM_V && bc.n_electrodes > 0 && !bc.pot_dirichlet[PFD_BOTTOM] && n64 > 0) n64 = c->planes;
    c->n64[f] = n64;
  }
  for (int f = 0; f < 5 && !e; ++f) e = up(c->d_anorm[f], an[f].data(), 8 * c->planes);
  if (!e) e = hipMemsetAsync(c->d_gate, 0, 64, c->stream);
  if (!e) e = hipMemsetAsync(c->d_rstat, 0, 8 * 20, c->stream);
  c->refine_max = prob->refine_max > 0 ? prob->refine_max : PFD_REFINE_MAX_DEFAULT;
  c->refine_tol = prob->refine_tol > 0 ? prob->refine_tol : PFD_REFINE_TOL_DEFAULT;
  if (!e) for (int s = 0; s < 4; ++s) { e = up(c->bm_side[s], bs[s].data(), 8 * c->Ng); if (e) break; }
  if (!e) e = up(c->bm_open, bo.data(), 8 * c->Ng);
  if (!e) e = up(c->bm_wall, bw.data(), 8 * c->Ng);
  if (!e) e = up(c->Mdiag, Md.data(), 8 * c->Ng);
  if (!e) e = up(c->d_hx, hx.data(), 8 * m.nx);
  if (!e) e = up(c->d_hy, hy.data(), 8 * m.ny);
  if (!e) e = up(c->d_w, c->w.data(), 8 * (K + 1));
  if (!e) e = up(c->d_D, c->D.data(), 8 * (K + 1) * (K + 1));
  if (!e) e = up(c->d_beta2, c->beta2.data(), 8 * c->planes);
  if (!e) e = up(c->d_betad, c->betad.data(), 8 * c->planes);
  for (int f = 0; f < 5 && !e; ++f)
    for (int k = 0; k < 3 && !e; ++k) e = up(c->fam[f].dshift + k * c->planes, c->fam[f].hshift.data(), 8 * c->planes);
  if (c->is3d && !e) {
    const size_t nz2 = 8 * (size_t)m.nz * m.nz;
    e = up(c->Wf, Wf.data(), nz2);
    if (!e) e = up(c->Wi, Wi.data(), nz2);
    if (!e) e = up(c->Wd, Wd.data(), nz2);
    if (!e) e = up(c->Dz, Dz.data(), nz2);
    std::vector<double> tr(m.nz / 2 + 1), ti(m.nz / 2 + 1);
    for (int k = 0; k <= m.nz / 2; ++k) {
      tr[k] = std::cos(2.0 * M_PI * k / m.nz);
      ti[k] = -std::sin(2.0 * M_PI * k / m.nz);
    }
    if (!e) e = up(c->twr, tr.data(), 8 * (m.nz / 2 + 1));
    if (!e) e = up(c->twi, ti.data(), 8 * (m.nz / 2 + 1));
    c->zlg = 0;
    if ((m.nz & (m.nz - 1)) == 0 && m.nz >= 4 && m.nz <= 256)   // FFT kernels for 4..256 planes
      while ((1 << c->zlg) < m.nz) ++c->zlg;
    for (int f : {F_UX, F_UY, F_UZ, F_P, F_PHI, F_PSI, F_V})
      for (int l = 0; l < 2 && !e; ++l) e = hipMemsetAsync(c->spec[f][l], 0, 8 * Pg, c->stream);
    for (int s : {PFD_SRC_VD, PFD_SRC_F2, PFD_SRC_WX, PFD_SRC_WY, PFD_SRC_WZ})
      if (!e) e = hipMemsetAsync(c->srcS[s], 0, 8 * Pg, c->stream);
  }
  // zero every field and source
  for (int f = 0; f < F_NSTATE && !e; ++f)
    for (int l = 0; l < 2 && !e; ++l) e = hipMemsetAsync(c->fld[f][l], 0, 8 * Pg, c->stream);
  for (int s = 0; s < PFD_NSRC && !e; ++s) e = hipMemsetAsync(c->src[s], 0, 8 * Pg, c->stream);
  if (!e) e = hipMemsetAsync(zero, 0, 8 * Pg, c->stream);
  if (!e) e = hipMemsetAsync(c->d_status, 0, 64, c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) { g_create_err = std::string("HIP error in create: ") + hipGetErrorString(e); delete c; return PFD_EHIP; }

  Geo& g = c->geo;
  g.K = K; g.n = K + 1; g.nq = c->nq; g.nx = m.nx; g.ny = m.ny; g.Nx = c->Nx; g.Ny = c->Ny;
  g.periodic = per ? 1 : 0; g.planes = c->planes; g.Ng = c->Ng; g.Nl = c->Nl;
  g.ppw = std::max(1, std::min(c->planes, 256 / c->nq));
  g.hx = c->d_hx; g.hy = c->d_hy; g.w = c->d_w; g.D = c->d_D;
  for (int s = 0; s < 4; ++s) {
    g.bm_side[s] = c->bm_side[s];
    g.side_type[s] = (per && s >= PFD_LEFT) ? -1 : bc.side_type[s];
  }
  c->zero_buf = zero;
  // ---- electrode gap nodes of the potential operator (Schur complement, FP64)
  if (bc.n_electrodes > 0 && !bc.pot_dirichlet[PFD_BOTTOM]) {
    const Dir1D& vx = c->dirs[c->fam[PFD_FAM_V].ix];
    const Dir1D& vy = c->dirs[c->fam[PFD_FAM_V].iy];
    Elec& E = c->elec;
    E.ebot.assign(c->Nx, 0);
    const double tol = 1e-10 * (m.xb[m.nx] - m.xb[0]);
    for (int ix = 0; ix < c->Nx; ++ix) {
      const double x = vx.coord[ix];
      for (int i = 0; i < bc.n_electrodes; ++i)
        if (x >= bc.electrode_x0[i] - tol && x <= bc.electrode_x1[i] + tol) E.ebot[ix] = 1;
      if (vx.dir[ix]) E.ebot[ix] = 1;
    }
    std::vector<int> gapidx(c->Nx, -1);
    for (int ix = 0; ix < c->Nx; ++ix)
      if (!E.ebot[ix]) {
        gapidx[ix] = (int)E.gap.size();
        E.gap.push_back(ix);
      }
    E.ng = (int)E.gap.size();
    if (E.ng > 0) {
      E.d_gap = (int*)carve(c, sizeof(int) * E.ng);
      E.d_gapidx = (int*)carve(c, sizeof(int) * c->Nx);
      E.d_ebot = (unsigned char*)carve(c, c->Nx);
      E.d_Sinv = D((long)c->planes * E.ng * E.ng);
      E.d_dG = D((long)c->planes * E.ng);
      if (!E.d_gap || !E.d_gapidx || !E.d_ebot || !E.d_Sinv || !E.d_dG) {
        g_create_err = "workspace too small (electrodes)"; delete c; return PFD_ENOMEM;
      }
      std::vector<double> all((size_t)c->planes * E.ng * E.ng), Sinv;
      double last_shift = -1.0;
      for (int p = 0; p < c->planes; ++p) {
        const double sh = c->fam[PFD_FAM_V].hshift[p];
        if (p == 0 || sh != last_shift) electrode_schur_inverse(vx, vy, E.gap, K, sh, Sinv);
        last_shift = sh;
        std::copy(Sinv.begin(), Sinv.end(), all.begin() + (size_t)p * E.ng * E.ng);
      }
      e = hipMemcpy(E.d_gap, E.gap.data(), sizeof(int) * E.ng, hipMemcpyHostToDevice);
      if (!e) e = hipMemcpy(E.d_gapidx, gapidx.data(), sizeof(int) * c->Nx, hipMemcpyHostToDevice);
      if (!e) e = hipMemcpy(E.d_ebot, E.ebot.data(), c->Nx, hipMemcpyHostToDevice);
      if (!e) e = hipMemcpy(E.d_Sinv, all.data(), 8 * all.size(), hipMemcpyHostToDevice);
      if (e) { g_create_err = std::string("HIP error in create: ") + hipGetErrorString(e); delete c; return PFD_EHIP; }
    }
  }
  for (int f = 0; f < 5; ++f) {
    const Dir1D& dx = c->dirs[c->fam[f].ix];
    const Dir1D& dy = c->dirs[c->fam[f].iy];
    c->lift[f] = Lift{dx.dK0, dx.dKN, dy.dK0, dy.dKN, dx.dM1, dy.dM1, dx.dKb, dx.ddir, dy.ddir,
                      (f == PFD_FAM_V && c->elec.ng > 0) ? c->elec.d_ebot : nullptr};
  }
  e = autotune(c);
  if (e) { g_create_err = std::string("HIP error in create (autotune): ") + hipGetErrorString(e); delete c; return PFD_EHIP; }
  *out = c;
  return PFD_OK;
}

static void drop_graphs(pfd_ctx* c);

extern "C" void pfd_destroy(pfd_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

extern "C" pfd_status pfd_get_dims(const pfd_ctx* c, int* Nx, int* Ny, int* planes) {
  if (!c) return PFD_EINVAL;
  if (Nx) *Nx = c->Nx;
  if (Ny) *Ny = c->Ny;
  if (planes) *planes = c->planes;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_coords(const pfd_ctx* c, double* x, double* y, double* z) {
  if (!c) return PFD_EINVAL;
  const Dir1D& DX = c->dirs[c->fam[0].ix];
  const Dir1D& DY = c->dirs[c->fam[0].iy];
  if (x) std::memcpy(x, DX.coord.data(), sizeof(double) * c->Nx);
  if (y) std::memcpy(y, DY.coord.data(), sizeof(double) * c->Ny);
  if (z)
    for (int p = 0; p < c->planes; ++p)
      z[p] = c->is3d ? p * c->prob.mesh.lz / c->prob.mesh.nz : 0.0;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_diag(pfd_ctx* c, pfd_diag* d) {
  if (!c || !d) return PFD_EINVAL;
  const Par& P = c->par;
  double v[10] = {P.gamma0, P.S, P.alpha, P.c_psi, P.c_phi, P.eps0, P.rho0, P.nu_m, P.c_u, 0.0};
  std::memcpy(d->derived, v, sizeof(v));
  int st[2] = {0, 0};
  double rs[20];
  hipError_t e = hipMemcpyAsync(st, c->d_status, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipMemcpyAsync(rs, c->d_rstat, sizeof(rs), hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipMemsetAsync(c->d_status + 1, 0, sizeof(int), c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  if (e) { c->err = hipGetErrorString(e); return PFD_EHIP; }
  d->nonfinite = st[0] & 1;
  d->unconverged = st[1];
  d->last_residual = 0.0;
  if (c->prob.precision == PFD_REFINED_FP32)
    for (int f = 0; f < 5; ++f)
      if (c->n64[f] < c->planes) d->last_residual = std::max(d->last_residual, rs[4 * f + 1]);
  d->steps = c->steps;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_refine_stats(pfd_ctx* c, pfd_refine_stats* out, int reset) {
  if (!c || !out) return PFD_EINVAL;
  double rs[20];
  HIPCHK(hipMemcpyAsync(rs, c->d_rstat, sizeof(rs), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const bool refined = c->prob.precision == PFD_REFINED_FP32;
  for (int f = 0; f < 5; ++f) {
    pfd_refine_stats& o = out[f];
    o.n_fp64_planes = refined ? c->n64[f] : c->planes;
    o.last_corrections = (int)rs[4 * f];
    o.last_eta = rs[4 * f + 1];
    o.max_corrections = (int)rs[4 * f + 2];
    o.failures = (long)rs[4 * f + 3];
    o.kappa_min = c->kappa_min[f];
    o.kappa_max = c->kappa_max[f];
  }
  if (reset) {
    for (int f = 0; f < 5; ++f) rs[4 * f + 2] = rs[4 * f + 3] = 0.0;
    HIPCHK(hipMemcpyAsync(c->d_rstat, rs, sizeof(rs), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return PFD_OK;
}

// Status words of a context after stream-ordered work: [0] bit 0 non-finite, [1] bit f a
// family-f refined solve missed the stop rule.  Reads both and clears [1].  Synchronises.
hipError_t pfd::read_status(pfd_ctx* c, int* st) {
  hipError_t e = hipMemcpyAsync(st, c->d_status, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (!e) e = hipMemsetAsync(c->d_status + 1, 0, sizeof(int), c->stream);
  if (!e) e = hipStreamSynchronize(c->stream);
  return e;
}

// the PFD_ENOCONV message of a family mask
std::string pfd::unconverged_msg(int mask) {
  static const char* nm[5] = {"V", "psi", "phi", "P", "u"};
  std::string m = "iterative refinement missed its stop rule (family";
  for (int f = 0; f < 5; ++f)
    if (mask & (1 << f)) m += std::string(" ") + nm[f];
  return m + ")";
}

static double* field_ptr(pfd_ctx* c, int f, int level) {
  if (f < 0 || f >= PFD_NFIELDS) return nullptr;
  const bool two = (f <= PFD_V);
  if (level != 0 && !(two && level == -1)) return nullptr;
  if (f >= PFD_EX) return c->fld[f][0];
  return c->fld[f][level == 0 ? c->cur : 1 - c->cur];
}

extern "C" pfd_status pfd_set_field(pfd_ctx* c, int f, int level, const double* src, int on_device) {
  if (!c || !src) return PFD_EINVAL;
  double* dst = field_ptr(c, f, level);
  if (!dst) { c->err = "bad field or level"; return PFD_EINVAL; }
  const size_t bytes = sizeof(double) * c->planes * c->Ng;
  hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, k, c->stream));
  if (level == 0 && f <= PFD_V) {
    double* old = field_ptr(c, f, -1);
    HIPCHK(hipMemcpyAsync(old, src, bytes, k, c->stream));
  }
  if (c->is3d && f <= PFD_V) {  // spectral copies (both levels when level 0 was set)
    const int lv = (level == 0) ? c->cur : 1 - c->cur;
    HIPCHK(to_spectral(c, c->fld[f][lv], c->spec[f][lv]));
    if (level == 0) HIPCHK(to_spectral(c, c->fld[f][lv], c->spec[f][1 - lv]));
  }
  if (!on_device) HIPCHK(hipStreamSynchronize(c->stream));
  forget_rhs(c);
  c->failed = 0;
  c->steps = 0;
  HIPCHK(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
  return PFD_OK;
}

extern "C" pfd_status pfd_get_field(pfd_ctx* c, int f, int level, double* dst, int on_device) {
  if (!c || !dst) return PFD_EINVAL;
  double* src = field_ptr(c, f, level);
  if (!src) { c->err = "bad field or level"; return PFD_EINVAL; }
  const size_t bytes = sizeof(double) * c->planes * c->Ng;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  if (!on_device) HIPCHK(hipStreamSynchronize(c->stream));
  return PFD_OK;
}

extern "C" pfd_status pfd_set_source(pfd_ctx* c, int s, const double* src, int on_device) {
  if (!c || s < 0 || s >= PFD_NSRC) return PFD_EINVAL;
  const size_t bytes = sizeof(double) * c->planes * c->Ng;
  c->src_dirty[s] = 1;
  forget_rhs(c);
  if (!src) {
    HIPCHK(hipMemsetAsync(c->src[s], 0, bytes, c->stream));
  } else {
    HIPCHK(hipMemcpyAsync(c->src[s], src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          c->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(c->stream));
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_init_potential(pfd_ctx* c, double tol, int max_iter, int* iters) {
  if (!c) return PFD_EINVAL;
  if (max_iter < 1) { c->err = "max_iter must be >= 1"; return PFD_EINVAL; }
  forget_rhs(c);
  double* A = c->fld[F_V][c->cur];
  double* B = c->fld[F_V][1 - c->cur];
  int it = 0;
  bool conv = false;
  for (it = 1; it <= max_iter; ++it) {
    HIPCHK(c->is3d ? potential_iteration_3d(c, A, B) : potential_iteration(c, A, B));
    double h[2];
    HIPCHK(max_abs_diff(c, A, B, h));
    std::swap(A, B);  // A = newest
    if (!std::isfinite(h[0])) { c->err = "non-finite potential"; return PFD_ENONFINITE; }
    if (h[0] <= tol * std::max(1.0, h[1])) { conv = true; break; }
  }
  if (it > max_iter) it = max_iter;
  const size_t bytes = sizeof(double) * c->planes * c->Ng;
  double* cur = c->fld[F_V][c->cur];
  if (A != cur) HIPCHK(hipMemcpyAsync(cur, A, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(c->fld[F_V][1 - c->cur], cur, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->is3d) {
    HIPCHK(to_spectral(c, cur, c->spec[F_V][c->cur]));
    HIPCHK(to_spectral(c, cur, c->spec[F_V][1 - c->cur]));
  }
  HIPCHK(update_E(c));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (iters) *iters = it;
  if (!conv) { c->err = "potential fixed point did not converge"; return PFD_ENOCONV; }
  return PFD_OK;
}

// recycling of the right sides (refined path): state kept on the host, outside any graph
void pfd::forget_rhs(pfd_ctx* c) {
  for (int& h : c->bhist) h = 0;
}
void pfd::begin_step(pfd_ctx* c, int eq) {
  // the recycled first residual needs the two previous solves of every refined family to have
  // met the stop rule (tested on the device; a miss is reported as PFD_ENOCONV)
  bool ok = c->prob.precision == PFD_REFINED_FP32;
  for (int f = 0; f < 5; ++f)
    if ((!eq || f == PFD_FAM_V || f == PFD_FAM_PSI || f == PFD_FAM_PHI) && warm_start(c, f))
      ok = ok && c->bhist[f] >= 2;
  c->rec_on = ok;
}
void pfd::end_step(pfd_ctx* c, int eq) {
  for (int f = 0; f < 5; ++f) {
    const bool solved = !eq || f == PFD_FAM_V || f == PFD_FAM_PSI || f == PFD_FAM_PHI;
    c->bhist[f] = solved ? std::min(2, c->bhist[f] + 1) : 0;
  }
  c->rec_on = false;
}
static hipError_t one_step_launch(pfd_ctx* c, int eq);

static void drop_graphs(pfd_ctx* c) {
  ++c->graph_gen;   // a batch holding this context's launches recaptures
  for (auto& row : c->gexec)
    for (auto& g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// one step: eager launches, or the replay of a captured graph of the same launches
static hipError_t one_step(pfd_ctx* c, int eq) {
  begin_step(c, eq);
  hipError_t es = one_step_launch(c, eq);
  end_step(c, eq);
  return es;
}

// one step's launches (begin_step decided whether it recycles the right sides)
static hipError_t one_step_launch(pfd_ctx* c, int eq) {
  const bool refined = c->prob.precision == PFD_REFINED_FP32;
  // graphs hold the recycling form of a refined step only (the two steps before it run eagerly)
  if (!c->use_graph || c->prof_on || (refined && !c->rec_on))
    return c->is3d ? step_once_3d(c, eq) : step_once(c, eq);
  if (c->is3d) refresh_spectral_sources(c);  // host-decided transforms stay outside the graph
  const int cur = c->cur;
  hipGraphExec_t& ex = c->gexec[cur][eq ? 1 : 0];
  if (!ex) {
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e) { c->stream = user; return e; }
    hipError_t es = c->is3d ? step_once_3d(c, eq) : step_once(c, eq);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &gr);
    c->stream = user;
    c->cur = cur;
    if (!e) e = es;
    if (!e) e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (gr) (void)hipGraphDestroy(gr);
    if (e) { ex = nullptr; return e; }
  }
  hipError_t e = hipGraphLaunch(ex, c->stream);
  if (e) return e;
  c->cur = 1 - cur;
  return hipSuccess;
}

extern "C" pfd_status pfd_get_mass_weights(pfd_ctx* c, double* w) {
  if (!c || !w) return PFD_EINVAL;
  HIPCHK(hipMemcpyAsync(w, c->Mdiag, sizeof(double) * c->Ng, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->is3d)
    for (long i = 0; i < c->Ng; ++i) w[i] *= c->prob.mesh.lz / c->planes;
  return PFD_OK;
}

extern "C" pfd_status pfd_update_params(pfd_ctx* c, const pfd_params* q) {
  if (!c || !q) return PFD_EINVAL;
  const pfd_params& o = c->prob.par;
  if (q->rho1 != o.rho1 || q->rho2 != o.rho2 || q->mu1 != o.mu1 || q->mu2 != o.mu2 || q->lambda != o.lambda ||
      q->eta != o.eta || q->gamma1 != o.gamma1 || q->dt != o.dt || q->bdf_order != o.bdf_order || q->S != o.S ||
      q->nu_m != o.nu_m) {
    c->err = "only eps1, eps2 and theta_s_deg may change after create";
    return PFD_EINVAL;
  }
  if (!(q->eps1 > 0.0) || !(q->eps2 > 0.0)) { c->err = "permittivities must be positive"; return PFD_EINVAL; }
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);   // kernel arguments change
  forget_rhs(c);    // and the potential's operator may
  c->prob.par = *q;
  Par& P = c->par;
  P.eps1 = q->eps1;
  P.eps2 = q->eps2;
  P.eps0 = std::max(q->eps1, q->eps2);
  P.cos_theta = std::cos(q->theta_s_deg * M_PI / 180.0);
  return PFD_OK;
}

extern "C" pfd_status pfd_set_solver_variant(pfd_ctx* c, int variant) {
  if (!c || variant < -1 || variant > 2) return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  if (variant < 0)
    HIPCHK(autotune(c));
  else
    c->fdm_variant = variant;
  return PFD_OK;
}

extern "C" pfd_status pfd_set_gemm_config(pfd_ctx* c, int site, int cfg) {
  if (!c || site < -1 || site >= PFD_GS_N || cfg < 0) return PFD_EINVAL;
  if (cfg >= PFD_GEMM_NCFG && !(cfg == PFD_ZFFT_CFG && site == PFD_GS_Z && c->zlg > 0)) return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  for (int s = 0; s < PFD_GS_N; ++s)
    if (site < 0 || s == site) c->gemm_cfg[s][0] = c->gemm_cfg[s][1] = cfg;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_gemm_config(const pfd_ctx* c, int* cfg, double* us) {
  if (!c) return PFD_EINVAL;
  const int ti = (c->prob.precision == PFD_REFINED_FP32) ? 0 : 1;
  for (int s = 0; s < PFD_GS_N; ++s) {
    const int t = (s == PFD_GS_Z) ? 1 : ti;
    if (cfg) cfg[s] = c->gemm_cfg[s][t];
    if (us) {
      for (int k = 0; k < PFD_GEMM_NCFG; ++k) us[s * (PFD_GEMM_NCFG + 1) + k] = c->gemm_us[s][t][k];
      us[s * (PFD_GEMM_NCFG + 1) + PFD_GEMM_NCFG] = (s == PFD_GS_Z) ? c->zfft_us : 0.0;
    }
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_get_tuning(const pfd_ctx* c, int* vals, int n, int* count) {
  if (!c || n < 0 || (n > 0 && !vals)) return PFD_EINVAL;
  int t[2 * PFD_GS_N + 5];
  int k = 0;
  for (int s = 0; s < PFD_GS_N; ++s) {
    t[k++] = c->gemm_cfg[s][0];
    t[k++] = c->gemm_cfg[s][1];
  }
  t[k++] = c->fdm_variant;
  t[k++] = c->resid_variant;
  t[k++] = c->mid_tn;
  t[k++] = c->p4_tg;
  t[k++] = c->p1_srp;
  for (int i = 0; i < k && i < n; ++i) vals[i] = t[i];
  if (count) *count = k;
  return PFD_OK;
}

extern "C" pfd_status pfd_set_tuning(pfd_ctx* c, const int* vals, int n) {
  if (!c || !vals || n != 2 * PFD_GS_N + 5) return PFD_EINVAL;
  for (int s = 0; s < PFD_GS_N; ++s)
    for (int t = 0; t < 2; ++t) {
      const int cfg = vals[2 * s + t];
      if (cfg < 0 || (cfg >= PFD_GEMM_NCFG && !(cfg == PFD_ZFFT_CFG && s == PFD_GS_Z && c->zlg > 0)))
        return PFD_EINVAL;
    }
  const int* v = vals + 2 * PFD_GS_N;
  if (v[0] < 0 || v[0] > 2 || v[1] < 0 || v[1] > 3 || v[2] < 1 || v[2] > 2 || v[3] < 0 || v[3] > 6 || v[4] < 0 ||
      v[4] > 1)
    return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  for (int s = 0; s < PFD_GS_N; ++s)
    for (int t = 0; t < 2; ++t) c->gemm_cfg[s][t] = vals[2 * s + t];
  c->fdm_variant = v[0];
  c->resid_variant = v[1];
  c->mid_tn = c->mid_best_tn = v[2];
  c->p4_tg = v[3];
  c->p1_srp = v[4];
  return PFD_OK;
}

extern "C" pfd_status pfd_set_residual_variant(pfd_ctx* c, int variant) {
  if (!c || variant < 0 || variant > 3) return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->resid_variant = variant;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_residual_variant(const pfd_ctx* c, int* variant, double* us) {
  if (!c) return PFD_EINVAL;
  if (variant) *variant = c->resid_variant;
  if (us)
    for (int v = 0; v < 3; ++v) us[v] = c->resid_us[v];
  return PFD_OK;
}

extern "C" pfd_status pfd_get_solver_variant(const pfd_ctx* c, int* variant, double* us) {
  if (!c) return PFD_EINVAL;
  if (variant) *variant = c->fdm_variant;
  if (us)
    for (int v = 0; v < 3; ++v) us[v] = c->fdm_us[v];
  return PFD_OK;
}

extern "C" pfd_status pfd_set_graph(pfd_ctx* c, int on) {
  if (!c) return PFD_EINVAL;
  if (on && !c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (!on) {
    HIPCHK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
  }
  c->use_graph = on ? 1 : 0;
  return PFD_OK;
}

extern "C" pfd_status pfd_step_async(pfd_ctx* c, int nsteps, int equilibrium) {
  if (!c || nsteps < 0) return PFD_EINVAL;
  if (c->failed) { c->err = "context failed earlier; set the fields again"; return PFD_ESTATE; }
  for (int i = 0; i < nsteps; ++i) HIPCHK(one_step(c, equilibrium));
  c->steps += nsteps;
  return PFD_OK;
}

extern "C" pfd_status pfd_get_stats(pfd_ctx* c, pfd_stats* out) {
  if (!c || !out) return PFD_EINVAL;
  const int ninst = c->is3d ? 1 : c->planes;
  std::vector<double> h((size_t)ninst * 8);
  HIPCHK(stats(c, h.data()));
  for (int i = 0; i < ninst; ++i) {
    const double* o = &h[(size_t)i * 8];
    pfd_stats& s = out[i];
    s.mass = o[0];
    s.kinetic = o[1];
    s.mixing = o[2];
    s.electric = o[3];
    s.wall = o[4];
    s.total = o[5];
    s.phi_max_abs = o[6];
    s.nonfinite = o[7] > 0.0 ? 1 : 0;
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_march_to_equilibrium(pfd_ctx* c, double tol, long max_steps, long* steps,
                                               double* residual) {
  if (!c || !(tol >= 0.0) || max_steps < 1) return PFD_EINVAL;
  if (c->failed) { c->err = "context failed earlier; set the fields again"; return PFD_ESTATE; }
  long n = 0;
  double r = 0.0;
  bool conv = false;
  while (n < max_steps) {
    HIPCHK(one_step(c, 1));
    ++n;
    ++c->steps;
    double h[2];
    HIPCHK(max_abs_diff(c, c->fld[F_PHI][c->cur], c->fld[F_PHI][1 - c->cur], h));
    int st[2] = {0, 0};
    HIPCHK(read_status(c, st));
    r = h[0];
    if ((st[0] & 1) || !std::isfinite(r)) {
      c->failed = 1;
      c->err = "non-finite value in the state";
      if (steps) *steps = n;
      if (residual) *residual = r;
      return PFD_ENONFINITE;
    }
    if (st[1]) {
      c->err = unconverged_msg(st[1]);
      if (steps) *steps = n;
      if (residual) *residual = r;
      return PFD_ENOCONV;
    }
    if (r <= tol) { conv = true; break; }
  }
  if (steps) *steps = n;
  if (residual) *residual = r;
  if (!conv) { c->err = "equilibrium tolerance not reached"; return PFD_ENOCONV; }
  return PFD_OK;
}

extern "C" pfd_status pfd_step(pfd_ctx* c, int nsteps, int equilibrium) {
  pfd_status s = pfd_step_async(c, nsteps, equilibrium);
  if (s != PFD_OK) return s;
  int st[2] = {0, 0};
  HIPCHK(read_status(c, st));
  if (st[0] & 1) {
    c->failed = 1;
    c->err = "non-finite value in the state";
    return PFD_ENONFINITE;
  }
  if (st[1]) {
    c->err = unconverged_msg(st[1]);
    return PFD_ENOCONV;
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_solve(pfd_ctx* c, int fam, const double* b, double* x) {
  if (!c || !b || !x || fam < 0 || fam > 4) return PFD_EINVAL;
  HIPCHK(solve(c, fam, b, x, 1, 1, nullptr, false));
  return PFD_OK;
}

extern "C" pfd_status pfd_apply(pfd_ctx* c, int fam, const double* x, double* y) {
  if (!c || !x || !y || fam < 0 || fam > 4) return PFD_EINVAL;
  HIPCHK(apply(c, fam, x, y, 1));
  return PFD_OK;
}

extern "C" pfd_status pfd_profile_enable(pfd_ctx* c, int on) {
  if (!c) return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->prof_on = on ? 1 : 0;
  c->ev_used = 0;
  c->prof_rec.clear();
  for (int k = 0; k < PFD_PROF_NCLASS; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_profile_read(pfd_ctx* c, int cls, double* total_ms, long* launches) {
  if (!c || cls < 0 || cls >= PFD_PROF_NCLASS) return PFD_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (const auto& r : c->prof_rec) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[r.second], c->ev_pool[r.second + 1]));
    c->prof_ms[r.first] += ms;
    c->prof_n[r.first] += 1;
  }
  c->prof_rec.clear();
  c->ev_used = 0;
  if (total_ms) *total_ms = c->prof_ms[cls];
  if (launches) *launches = c->prof_n[cls];
  return PFD_OK;
}

extern "C" pfd_status pfd_profile_replay(pfd_ctx* c, int cls, int reps, double* avg_us) {
  if (!c || !avg_us || reps < 1) return PFD_EINVAL;
  if (cls != PFD_PROF_GEMM32 && cls != PFD_PROF_GEMM64 && cls != PFD_PROF_RESID) {
    c->err = "replay supports the GEMM and residual classes";
    return PFD_EINVAL;
  }
  HIPCHK(replay(c, cls, reps, avg_us));
  return PFD_OK;
}
