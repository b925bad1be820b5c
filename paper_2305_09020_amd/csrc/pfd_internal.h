// Internal layout of a pfd context (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pfd.h"

#define PFD_KMAX 16        // array bounds of the 1D tables
#define PFD_KMAX_STEP 15   // highest order accepted: (K+1)^2 <= 256 element nodes per work-group
#define PFD_NMAX 320  // max nodes per direction handled by the solve kernels
#define PFD_STAT_NB 32  // blocks per instance of the diagnostics reduction
#define PFD_GEMM_NCFG 16  // tile configurations of the batched GEMM
// GEMM call sites tuned separately: the four fast-diagonalisation passes and the z transform
enum { PFD_GS_P1 = 0, PFD_GS_P2, PFD_GS_P3, PFD_GS_P4, PFD_GS_Z, PFD_GS_N };
#define PFD_ZFFT_CFG 16  // z-transform site only: the batched FFT instead of a GEMM

namespace pfd {

// One direction x one boundary-condition combination of the 1D operators.
struct Dir1D {
  int N = 0, nfree = 0;
  bool periodic = false;
  bool singular = false;            // no Dirichlet end: constants in the kernel
  std::vector<double> K1, M1, S, lam, coord;
  std::vector<char> dir;            // Dirichlet flag per node
  // device copies
  double *dS = nullptr, *dST = nullptr, *dlam = nullptr, *dKb = nullptr, *dM1 = nullptr;
  double *dK0 = nullptr, *dKN = nullptr;  // first and last columns of K1 (Dirichlet lifting)
  std::vector<double> Kb;            // banded transposed stiffness: Kb[(d+K)*N + i] = K1[i][i+d]
  float *fS = nullptr, *fST = nullptr;
  // S and S^T in MFMA fragment order (frag_layout), zero-padded to a multiple of 16
  double *dSw = nullptr, *dSTw = nullptr;
  float *fSw = nullptr, *fSTw = nullptr;
  unsigned char* ddir = nullptr;
};

struct Family {
  int ix = 0, iy = 0;               // indices into ctx dirs (x and y)
  double shift = 0.0;               // c_f (plus beta_p^2 per plane)
  double* dshift = nullptr;         // per-plane total shift (device)
  std::vector<double> hshift;       // per-plane total shift (host)
  bool any_singular = false;        // some plane has a singular operator
};

// geometry passed to element / nodal kernels by value
struct Geo {
  int K, n, nq, nx, ny, Nx, Ny, periodic, planes;
  int ppw;                          // planes per element work-group (ppw nq <= 256 when nq <= 256)
  long Ng, Nl;
  const double *hx, *hy, *w, *D;    // device
  const double *bm_side[4];         // per-side boundary mass (device, Ng)
  int side_type[4];                 // WALL/OPEN/-1 (absent, periodic)
};

// scalar parameters passed to kernels by value
struct Par {
  double rho1, rho2, mu1, mu2, eps1, eps2, lam, eta, gamma1, dt;
  double gamma0, S, alpha, c_psi, c_phi, eps0, rho0, nu_m, c_u;
  double cos_theta;
  double cs_n, cs_o, ch_n, ch_o;    // xi* = cs_n xi^n + cs_o xi^{n-1}; xi^ likewise
};

enum { F_UX = 0, F_UY, F_UZ, F_P, F_PHI, F_PSI, F_V, F_EX, F_EY, F_EZ, F_E2, F_NSTATE };

// Dirichlet lifting data of one solve family (device pointers).  ebot (potential family with
// partial electrode segments only): 1 on bottom-row nodes that are Dirichlet (electrodes),
// 0 on the gap nodes between them, which are unknowns although diry[0] marks the base
// operator's bottom row as Dirichlet.
struct Lift {
  const double *Kx0, *KxN, *Ky0, *KyN, *Mx, *My, *KxB;
  const unsigned char *dirx, *diry, *ebot;
  // FP32-refined path, set per launch: the family's right side b^n of the previous step (the
  // slot written now holds b^{n-1}); the first residual is then b - (cs_n b^n + cs_o b^{n-1})
  const double* bprev = nullptr;
};

// gap-node Schur complement data of the potential family (electrode segments)
struct Elec {
  int ng = 0;                       // number of gap nodes on the bottom row
  std::vector<int> gap;             // their x indices
  std::vector<unsigned char> ebot;  // Nx flags: Dirichlet (electrode) bottom nodes
  int *d_gap = nullptr, *d_gapidx = nullptr;
  unsigned char* d_ebot = nullptr;
  double *d_Sinv = nullptr, *d_dG = nullptr;  // planes x ng x ng, planes x ng
};

// one recorded kernel launch (a context stepping in record mode, for a multi-instance batch):
// the kernel's multi-instance form, launch shape, and its packed arguments
struct RecLaunch {
  const void* fn = nullptr;
  unsigned grid[3] = {1, 1, 1}, block[3] = {1, 1, 1};
  size_t shm = 0, asize = 0, aalign = 1;
  std::vector<unsigned char> args;
};

}  // namespace pfd

struct pfd_ctx {
  pfd_problem prob;
  std::string err;
  hipStream_t stream = nullptr;
  int device = 0;                          // current device at pfd_create
  int Nx = 0, Ny = 0, planes = 0, is3d = 0;
  long Ng = 0, Nl = 0;
  int K = 0, n = 0, nq = 0;
  pfd::Par par{};
  pfd::Geo geo{};
  std::vector<double> xi, w, D;            // GLL rule
  std::vector<pfd::Dir1D> dirs;            // distinct 1D operators
  pfd::Family fam[5];
  pfd::Lift lift[5];
  pfd::Elec elec;
  double* Ybuf = nullptr;                  // base-operator correction (electrode solves)
  std::vector<double> beta2, betad;        // per plane (spectral packing in 3D)
  double *d_beta2 = nullptr, *d_betad = nullptr;
  // device buffers
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_used = 0;
  bool ws_fail = false;                    // some workspace carve did not fit
  double* fld[pfd::F_NSTATE][2] = {};     // state fields, two time levels
  int cur = 0;                             // index of level n
  int set_old[pfd::F_NSTATE] = {};         // level n-1 explicitly set
  double* src[PFD_NSRC] = {};
  double *Lb[7] = {}, *b[3] = {}, *r = nullptr, *U = nullptr, *Q2 = nullptr;
  // 3D (Fourier in z): packed DFT matrices, spectral state, temporaries
  double *Wf = nullptr, *Wi = nullptr, *Wd = nullptr, *Dz = nullptr;
  double *twr = nullptr, *twi = nullptr;   // FFT twiddles exp(-2 pi i k / nz), k < nz/2
  int zlg = 0;                             // log2(nz) when nz is a power of two, else 0
  double zfft_us = 0.0;                    // autotune timing of the FFT (us per transform)
  double* spec[pfd::F_NSTATE][2] = {};     // spectral copies of u, P, phi, psi, V (two levels)
  double *ph[5] = {}, *sp[5] = {}, *dz[6] = {};
  double* srcS[PFD_NSRC] = {};             // spectral Dirichlet data (VD, F2, WX, WY, WZ)
  int src_dirty[PFD_NSRC] = {};
  double *tmp = nullptr, *tmp2 = nullptr;  // solve intermediates (double or float)
  double* d_part = nullptr;                // per-plane partial sums
  double Mtot = 0.0;                       // sum of the mass matrix (area)
  double* zero_buf = nullptr;              // planes*Ng zeros (u = 0 of the equilibrium system)
  double *bm_side[4] = {}, *bm_open = nullptr, *bm_wall = nullptr, *Mdiag = nullptr;
  double *d_hx = nullptr, *d_hy = nullptr, *d_w = nullptr, *d_D = nullptr;
  int* d_status = nullptr;                 // [0] nonfinite flag
  double* d_stats = nullptr;               // block partials of the diagnostics
  double* d_red = nullptr;                 // reduction scratch (planes)
  // refinement of the FP32-refined path (convergence test of every FP64 residual)
  double* d_rpart = nullptr;               // block partials of the test: r^2, (||A_p|| x)^2
  long rpart_max = 0;                      // blocks the partial array holds
  int* d_gate = nullptr;                   // 1 once the current solve has converged
  double* d_rstat = nullptr;               // per family: corrections, backward error, max, failures
  double* d_anorm[5] = {};                 // per family and plane: bound of ||A_p||_2
  const int* gate = nullptr;               // gate the kernels being launched read (nullptr: none)
  double refine_tol = 0.0;                 // stop at ||r|| <= tol (||A|| ||x|| + ||b||)
  int refine_max = 0;                      // corrections before PFD_ENOCONV
  // precision ladder: per family the planes [0, n64) take FP64 corrections (singular or
  // ill-conditioned operators), the rest FP32 with refinement; condition estimates per family
  int n64[5] = {0, 0, 0, 0, 0};
  double kappa_min[5] = {}, kappa_max[5] = {};
  long steps = 0;
  int failed = 0;
  // hipGraph replay of whole steps: one executable per (parity of the current level, step kind)
  int use_graph = 0;
  // fast-diagonalisation kernels: 0 = four split-K GEMM passes, 1 = two fused strip kernels
  // (chosen by timing both at create)
  int fdm_variant = 1;
  int resid_variant = 1;                   // residual: 0 = per-node global reads, 1 = LDS tiles,
                                           // 2 = LDS tiles fused with the first FDM pass (refined),
                                           // 3 = per node with the order a runtime argument
  double resid_us[3] = {0.0, 0.0, 0.0};
  double fdm_us[3] = {0.0, 0.0, 0.0};      // autotune timings (us per correction)
  int mid_tn = 1, mid_best_tn = 1;         // column tiles per work-group of the fused middle passes
  int p4_tg = 0;                           // refined last pass: 0 = GEMM, 1..4 = k_p4 column tiles per
                                           // wave, 5 = k_srp (matrix resident in LDS), 6 = k_p4 one
                                           // tile with four-slice fragment chunks
  int p1_srp = 0;                          // refined first pass through k_srp
  int num_cu = 256, lds_max = 65536;       // device: compute units, LDS bytes a work-group may use
  long long hold_ticks = 50000;            // 0.5 ms of the device wall clock (autotuner's stream hold)
  // right sides of the step's solves per family and time level (u: three components), and how
  // many consecutive steps solved the family with them (the refined path recycles them for its
  // first residual once two are recorded: A x^n = b^n to the refinement's accuracy)
  double* bh[5][2] = {};
  int bhist[5] = {0, 0, 0, 0, 0};
  bool rec_on = false;                     // this step recycles (decided before the step)
  int gemm_cfg[PFD_GS_N][2] = {};          // tile configuration per (call site, FP32/FP64)
  double gemm_us[PFD_GS_N][2][PFD_GEMM_NCFG] = {};  // autotune timings per configuration
  hipStream_t cap_stream = nullptr;        // capture stream (the caller's may be the null stream)
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  unsigned long graph_gen = 0;             // bumped whenever captured launches become stale
  // per-kernel-class timing (pfd_profile_enable / pfd_profile_read)
  int prof_on = 0;
  // record mode: launches are appended here instead of being issued (nullptr: issue them)
  std::vector<pfd::RecLaunch>* rec = nullptr;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> prof_rec;   // (class, index of the start event)
  double prof_ms[PFD_PROF_NCLASS] = {};
  long prof_n[PFD_PROF_NCLASS] = {};
};

namespace pfd {
// timing scope around one launch (no-op unless profiling is enabled)
struct ProfScope {
  pfd_ctx* c;
  int cls;
  size_t i0;
  bool on;
  ProfScope(pfd_ctx* ctx, int k);
  ~ProfScope();
};

// set-up (pfd_setup.cpp)
void sym_eig(int n, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V);
void gll_rule(int K, std::vector<double>& x, std::vector<double>& w, std::vector<double>& D);
void build_dir1d(Dir1D& d, int ne, const double* bp, int K, bool periodic, bool dir_lo, bool dir_hi,
                 const std::vector<double>& xi, const std::vector<double>& w,
                 const std::vector<double>& D);
void electrode_schur_inverse(const Dir1D& dx, const Dir1D& dy, const std::vector<int>& gap, int K, double c,
                             std::vector<double>& Sinv);

// kernels (pfd_kernels.hip); all enqueue on ctx->stream
hipError_t solve(pfd_ctx* c, int fam, const double* b, double* x, int ncomp, int project, const double* r0,
                 bool r0_exact);
// the family's solves start from the extrapolated history: FP32-refined planes exist
inline bool warm_start(const pfd_ctx* c, int fam) {
  return c->prob.precision == PFD_REFINED_FP32 && c->n64[fam] < c->planes;
}
hipError_t apply(pfd_ctx* c, int fam, const double* x, double* y, int ncomp);
hipError_t step_once(pfd_ctx* c, int equilibrium);
hipError_t potential_iteration(pfd_ctx* c, const double* Vin, double* Vout);
hipError_t update_E(pfd_ctx* c);
hipError_t max_abs_diff(pfd_ctx* c, const double* a, const double* b, double* out_host2);
// per-instance diagnostics: out[inst*8 + q], q = mass, kinetic, mixing, electric, wall, total,
// max|phi|, non-finite count (host array of ninst*8; synchronises)
hipError_t stats(pfd_ctx* c, double* out);
hipError_t replay(pfd_ctx* c, int cls, int reps, double* avg_us);
hipError_t autotune(pfd_ctx* c);
hipError_t step_once_3d(pfd_ctx* c, int equilibrium);
// status words: st[0] bit 0 non-finite; st[1] refined families that missed the stop rule
// (cleared by the read); synchronises
hipError_t read_status(pfd_ctx* c, int* st);
std::string unconverged_msg(int mask);
// right-side recycling state of the refined path (host side): forget after any change of the
// state, sources or operators; begin_step decides whether a step recycles, end_step records it
void forget_rhs(pfd_ctx* c);
void begin_step(pfd_ctx* c, int eq);
void end_step(pfd_ctx* c, int eq);
void refresh_spectral_sources(pfd_ctx* c);
hipError_t potential_iteration_3d(pfd_ctx* c, const double* Vin, double* Vout);
hipError_t to_spectral(pfd_ctx* c, const double* phys, double* spec);
}  // namespace pfd
