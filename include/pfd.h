/*
 * pfd -- one time step of the decoupled phase-field scheme for two immiscible
 * dielectric fluids (Yang, Christov & Dong, arXiv 2305.09020) on an AMD
 * Instinct MI355X (gfx950).
 *
 * The library advances (u, P, phi, V) by Algorithm 1 (2D: C0 spectral elements,
 * Sec. 3.2.1, eqs. 54-59) or Algorithm 2 (3D: spectral elements in x-y times a
 * Fourier expansion in z, Sec. 3.2.2, eqs. 74-78).  Each step solves, in order,
 * V, E, psi, phi, P and u, every one with a constant coefficient matrix
 * (remark after Algorithm 2).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Floating point is IEEE binary64 (double) at the boundary.
 *  - Nodal arrays use the layout  value[(p * Ny + iy) * Nx + ix],
 *      Nx = nx*K + 1 - periodic_x,  Ny = ny*K + 1,
 *    p = plane: the z index j (z_j = j*Lz/Nz) in 3D, the instance index of a
 *    2D batch, 0 for a single 2D problem.  Node coordinates come from
 *    pfd_get_coords.
 *  - Memory: the caller owns every buffer.  Device memory for the whole
 *    context is ONE caller-allocated workspace (size from pfd_workspace_query);
 *    the library does not allocate device memory after pfd_create.  Host
 *    memory of the context (small tables) is allocated in pfd_create and freed
 *    by pfd_destroy.
 *  - Streams: every device operation is ordered on the hipStream_t given to
 *    pfd_create.  Entry points taking host buffers synchronise that stream
 *    before returning; entry points taking device buffers do not.
 *  - Errors: every call returns a pfd_status; pfd_last_error gives a message.
 *    A non-finite value detected in a step makes the context sticky-failed:
 *    further steps return PFD_ESTATE until a field is set again.
 *  - Threads: one context must not be used from two threads at once.
 */
#ifndef PFD_H
#define PFD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFD_OK = 0,
  PFD_EINVAL = 1,      /* bad argument or unsupported configuration            */
  PFD_ENOMEM = 2,      /* workspace too small                                  */
  PFD_EHIP = 3,        /* HIP runtime error                                    */
  PFD_ENONFINITE = 4,  /* a NaN/Inf appeared in the state during a step        */
  PFD_ENOCONV = 5,     /* a refined solve missed its stop rule within refine_max
                          corrections (pfd_step, pfd_step_async's later pfd_get_diag,
                          pfd_batch_step, pfd_march_to_equilibrium), or a fixed point /
                          equilibrium march missed its tolerance                 */
  PFD_ESTATE = 6,      /* context failed earlier or is not initialised         */
  PFD_ENOTIMPL = 7
} pfd_status;

/* fields readable/writable with pfd_get_field / pfd_set_field */
typedef enum {
  PFD_UX = 0, PFD_UY = 1, PFD_UZ = 2,   /* velocity u (eqs. 59, 78)            */
  PFD_P = 3,                            /* pressure P (eqs. 58, 77)            */
  PFD_PHI = 4,                          /* phase field phi (eqs. 57, 76)       */
  PFD_PSI = 5,                          /* auxiliary psi of eq. (44)           */
  PFD_V = 6,                            /* electric potential V (eqs. 54, 74)  */
  PFD_EX = 7, PFD_EY = 8, PFD_EZ = 9,   /* electric field E (eqs. 55, 78)      */
  PFD_NFIELDS = 10
} pfd_field;

/* source terms of the source-augmented system (Sec. 3.1, eqs. 27-33), nodal
 * values at t^{n+1}.  Volume sources: G (phase field), FX..FZ (momentum f),
 * FV (potential f_V).  Boundary sources (only values on the relevant boundary
 * nodes are read): G1 (n.grad of the chemical-potential bracket of eq. phia,
 * open and wall), G2 (n.grad phi, open), G3 (eq. phic, wall), F1X..F1Z
 * (du/dn, open), F2 (P, open), WX..WZ (u, wall), VD (V on the Dirichlet
 * electrode nodes).  Sources persist until replaced; a NULL pointer resets a
 * source to zero. */
typedef enum {
  PFD_SRC_G = 0, PFD_SRC_FX, PFD_SRC_FY, PFD_SRC_FZ, PFD_SRC_FV,
  PFD_SRC_G1, PFD_SRC_G2, PFD_SRC_G3, PFD_SRC_F1X, PFD_SRC_F1Y, PFD_SRC_F1Z,
  PFD_SRC_F2, PFD_SRC_WX, PFD_SRC_WY, PFD_SRC_WZ, PFD_SRC_VD,
  PFD_NSRC
} pfd_source;

/* precision of the constant-coefficient solves (the mixed-precision iterative refinement of
 * the constant matrices of Sec. 3, remark after Algorithm 2).
 * PFD_REFINED_FP32 applies, per solve, FP32 fast-diagonalisation corrections x += A~^{-1} r on
 * FP64 residuals r = b - A x until the normwise backward error of x (perturbations of A)
 *     eta = ||r||_2 / (||A||_2 ||x||_2)
 * (over the free nodes of all planes and stacked components, ||A_p||_2 bounded from the 1D
 * eigenvalues) is <= refine_tol, at most refine_max corrections; every FP64 residual is
 * tested on the device, and once a test passes the rest of the solve's kernels return at once
 * (so a captured step stays one graph).  A solve still above refine_tol after refine_max
 * corrections makes the stepping call return PFD_ENOCONV (the state is kept and valid, only
 * less accurate; the context does not fail).  Solves start from the extrapolated history;
 * once two consecutive steps have solved a family, the first residual is formed from the right
 * sides of those two steps (A x^n = b^n, to the stop rule) instead of a stencil pass, and the
 * first correction takes it untested.  That record is forgotten by pfd_set_field,
 * pfd_set_source, pfd_init_potential and pfd_update_params, and for P and u by an equilibrium
 * step (which does not solve them).
 * Precision ladder: at pfd_create each (family, plane) operator gets the condition estimate
 * kappa = (max lx + max ly + c_p) / (min lx + min ly + c_p) from its generalised 1D
 * eigenvalues; planes with kappa 2^-24 > 1/2 (the singular closed-box pressure and k = 0
 * pressure mode in particular) take one FP64 correction (a direct solve) instead.
 * pfd_get_refine_stats reports the estimates, the split and the corrections taken. */
typedef enum {
  PFD_PLAIN_FP64 = 0,   /* FP64 fast-diagonalisation solve                     */
  PFD_REFINED_FP32 = 1, /* FP32 solve + FP64 residual iterative refinement     */
  PFD_REFINED_BF16 = 2  /* not built: BF16 corrections were measured (bit-faithful
                           emulation on the benchmark operators) to need seven or
                           more corrections per solve against three in FP32, more
                           than their cheaper passes save; PFD_ENOTIMPL          */
} pfd_precision;

enum { PFD_WALL = 0, PFD_OPEN = 1, PFD_PERIODIC = 2 };
enum { PFD_BOTTOM = 0, PFD_TOP = 1, PFD_LEFT = 2, PFD_RIGHT = 3 };

/* solve families: the five constant operators (K + c M) of the step */
enum { PFD_FAM_V = 0, PFD_FAM_PSI = 1, PFD_FAM_PHI = 2, PFD_FAM_P = 3, PFD_FAM_U = 4 };

typedef struct {
  int nx, ny;            /* elements along x and y (tensor-product mesh)        */
  int K;                 /* element order, 2 <= K <= 15                         */
  const double* xb;      /* nx+1 increasing x breakpoints (host)                */
  const double* yb;      /* ny+1 increasing y breakpoints (host)                */
  int periodic_x;        /* 1: x = xb[0] and x = xb[nx] identified              */
  int nz;                /* 0: 2D; even >= 2: number of Fourier planes (3D)    */
  double lz;             /* period in z (3D)                                    */
  int nbatch;            /* 2D only: independent instances on this mesh (>=1)  */
} pfd_mesh;

typedef struct {
  double rho1, rho2;     /* densities (eq. interpolation)                       */
  double mu1, mu2;       /* dynamic viscosities                                 */
  double eps1, eps2;     /* permittivities                                      */
  double lambda;         /* mixing energy density (eq. double_well)             */
  double eta;            /* interface thickness                                 */
  double gamma1;         /* mobility                                            */
  double theta_s_deg;    /* static contact angle of eq. (theta_def), degrees    */
  double dt;             /* time step                                           */
  int bdf_order;         /* J = 1 or 2 (Sec. 3.1)                               */
  double S;              /* stabiliser; 0 -> eta^2 sqrt(4 gamma0/(lambda gamma1 dt)) */
  double nu_m;           /* 0 -> max(mu1,mu2)/min(rho1,rho2)                    */
} pfd_params;

typedef struct {
  int side_type[4];        /* PFD_WALL / PFD_OPEN per side (x sides ignored if periodic) */
  int pot_dirichlet[4];    /* 1: V Dirichlet on the whole side                   */
  /* Electrode segments on the bottom wall (eq. 21, and the gap condition
   * dV/dn = 0 between electrodes, Sec. 2): closed intervals [x0, x1] of x whose
   * bottom-row nodes carry Dirichlet V (its values come from PFD_SRC_VD, so each
   * electrode may hold its own voltage); the other bottom nodes are unknowns
   * with the natural condition.  Ends must lie on element edges, x0 < x1; with
   * periodic x a segment is taken in [xb[0], xb[nx]) (it covers the node at
   * xb[0] only if it starts there).  Host arrays, read during pfd_create only.
   * The gap nodes are eliminated through an FP64 capacitance (Schur complement)
   * matrix per Fourier mode, of size (gap nodes)^2, built at create time. */
  int n_electrodes;
  const double* electrode_x0;
  const double* electrode_x1;
} pfd_bcs;

typedef struct {
  pfd_mesh mesh;
  pfd_params par;
  pfd_bcs bc;
  int precision;         /* pfd_precision                                        */
  int refine_max;        /* PFD_REFINED_FP32: most corrections per solve, 0..64
                            (0 -> PFD_REFINE_MAX_DEFAULT)                         */
  double refine_tol;     /* PFD_REFINED_FP32: stop rule on eta, [0, 1)
                            (0 -> PFD_REFINE_TOL_DEFAULT)                         */
} pfd_problem;

#define PFD_REFINE_MAX_DEFAULT 3
#define PFD_REFINE_TOL_DEFAULT 1e-15

typedef struct pfd_ctx pfd_ctx;

typedef struct {
  double derived[10];    /* gamma0, S, alpha, c_psi, c_phi, eps0, rho0, nu_m, c_u, -  */
  double last_residual;  /* refined path: max over families of the backward error eta of
                            the last test of each family's last solve (0 on the plain path) */
  int nonfinite;         /* 1 if a non-finite value was seen                     */
  int unconverged;       /* bit f set: a family-f solve missed the stop rule since the last
                            pfd_step / pfd_get_diag / pfd_batch_step (cleared by this call) */
  long steps;            /* steps taken since the last pfd_set_field             */
} pfd_diag;

/* Iterative refinement record of one solve family (pfd_get_refine_stats). */
typedef struct {
  int n_fp64_planes;     /* planes [0, n) solved by one FP64 correction (precision ladder);
                            all planes on the plain FP64 path                    */
  int last_corrections;  /* FP32 corrections the last solve took                 */
  int max_corrections;   /* most corrections of one solve since the last reset   */
  long failures;         /* solves that missed the stop rule since the last reset */
  double last_eta;       /* backward error of the last test                      */
  double kappa_min, kappa_max;  /* condition estimates over the planes (inf: singular) */
} pfd_refine_stats;

/* Diagnostics of one instance (a 2D batch member, or the whole 3D field):
 * the mass int_h phi (conserved by eq. 16), and the discrete total energy of
 * eq. (14) term by term on the GLL quadrature: kinetic int 1/2 rho(phi)|u|^2;
 * mixing int F(phi, grad phi) of eq. (double_well) with the gradient part from
 * the assembled stiffness (plus (d_z phi)^2 in 3D); electric int 1/2 eps(phi)|E|^2
 * (D = eps E); wall int Theta(phi) over the wall sides, eq. (theta_def), with
 * gamma = sigma = 2 sqrt(2) lambda/(3 eta) and its constant term left out.
 * 3D sums include the z weight lz/nz. */
typedef struct {
  double mass;
  double kinetic, mixing, electric, wall, total;
  double phi_max_abs;    /* max |phi| over the instance                          */
  int nonfinite;         /* 1 if phi, |u|^2 or |E|^2 is not finite somewhere     */
} pfd_stats;

/* Refinement record of the five solve families (out[5], host; index = PFD_FAM_*), see
 * pfd_precision.  reset != 0 clears the corrections maximum and the failure count afterwards.
 * Synchronises the context's stream. */
pfd_status pfd_get_refine_stats(pfd_ctx* ctx, pfd_refine_stats* out, int reset);

/* Human-readable name of a status code.  Never NULL. */
const char* pfd_status_string(pfd_status s);

/* Message describing the last error on ctx (or on the most recent failed
 * pfd_create when ctx is NULL).  Valid until the next call on ctx. */
const char* pfd_last_error(const pfd_ctx* ctx);

/* Device bytes the context for *prob needs.  Host-only; validates prob
 * (PFD_EINVAL for: K outside [2,15], nx or ny < 1, non-increasing breakpoints,
 * dt <= 0, eta <= 0, odd or < 2 nz, nbatch < 1 or nbatch > 1 in 3D, an
 * electrode segment not on element edges, no V Dirichlet node at all). */
pfd_status pfd_workspace_query(const pfd_problem* prob, size_t* dev_bytes);

/* Build the context: GLL tables, 1D operators and their FP64 generalised
 * eigen-decompositions (Lynch-Rice-Thomas fast diagonalisation of the constant
 * matrices), electrode capacitance matrices, and device copies.  dev_ws is a
 * device buffer of at least dev_bytes from pfd_workspace_query, 256-byte
 * aligned, owned by the caller and kept alive until pfd_destroy.  stream is a
 * hipStream_t (NULL = default stream).  All fields start at zero. */
pfd_status pfd_create(const pfd_problem* prob, void* dev_ws, size_t dev_bytes,
                      void* stream, pfd_ctx** out);

/* Free host memory of ctx (the workspace stays the caller's).  NULL is a no-op. */
void pfd_destroy(pfd_ctx* ctx);

/* Nx, Ny and the number of planes (nz in 3D, nbatch in 2D). */
pfd_status pfd_get_dims(const pfd_ctx* ctx, int* Nx, int* Ny, int* planes);

/* Host copies of the 1D node coordinates: x[Nx], y[Ny], z[planes] (z may be
 * NULL; in 2D z is filled with zeros). */
pfd_status pfd_get_coords(const pfd_ctx* ctx, double* x, double* y, double* z);

/* Derived constants and diagnostics. */
pfd_status pfd_get_diag(pfd_ctx* ctx, pfd_diag* d);

/* Quadrature weights of one plane's nodes (host, Nx*Ny doubles): the discrete
 * integral of a field is sum over planes and nodes of w * f (the GLL mass
 * matrix; in 3D times lz/nz). */
pfd_status pfd_get_mass_weights(pfd_ctx* ctx, double* w);

/* Change the permittivities and the contact angle of a context (the constant
 * operators and their factors do not depend on them, so the set-up stays);
 * every other parameter must equal the current one (PFD_EINVAL otherwise).
 * Synchronises; drops captured graphs.  Used to march many equilibrium
 * problems on one context. */
pfd_status pfd_update_params(pfd_ctx* ctx, const pfd_params* par);

/* Kernels of the fast-diagonalisation solves: 0 = four batched GEMM passes
 * (tile configurations per pass from pfd_set_gemm_config), 1 = two fused
 * strip kernels (the strip intermediate stays in LDS), 2 = three launches:
 * the first and last passes as in 0, the two middle passes (along y, with the
 * division by the eigenvalue sums between them) fused in one kernel that keeps
 * a block of columns and its intermediate in LDS (falls back to 0 where that
 * block does not fit in 64 KB).  pfd_create times one velocity correction
 * with each in the context's solve precision and keeps the fastest; variant
 * -1 re-runs that autotuning.  All compute the same correction up to rounding
 * order.  Synchronises; drops captured graphs. */
pfd_status pfd_set_solver_variant(pfd_ctx* ctx, int variant);
/* Current variant and the autotuner's timings (us[3], microseconds per
 * correction of variants 0, 1 and 2; either may be NULL). */
pfd_status pfd_get_solver_variant(const pfd_ctx* ctx, int* variant, double* us);

/* Every choice of the autotuner (tile configurations per call site and precision, solver and
 * residual variants, block widths of the fused kernels) as an opaque list of integers, to copy
 * to another context of the same shapes so that both run the same kernels in the same order
 * (bit-identical results).  pfd_get_tuning writes min(n, count) values and the count (15) to
 * *count (either may be 0 / NULL); pfd_set_tuning takes exactly that count and rejects values
 * out of range (PFD_EINVAL).  Synchronises; drops captured graphs. */
pfd_status pfd_get_tuning(const pfd_ctx* ctx, int* vals, int n, int* count);
pfd_status pfd_set_tuning(pfd_ctx* ctx, const int* vals, int n);

/* Kernel of the FP64 residual b - (K + cM) x of the refinement: 0 = one
 * thread per node reading its 2(2K+1) band neighbours through the caches,
 * 1 = rows staged in LDS tiles (used when Nx <= 256 and the tile fits),
 * 2 = as 1 inside the refinement of the FP32-refined path, with the first
 * fast-diagonalisation pass (the rows times Sx) done in the same launch on
 * the matrix cores (not with solver variant 1, the electrode gap-node solve
 * or a singular operator's projection, where 1 is used), 3 = as 0 with the
 * element order a runtime argument rather than a compile-time one: one
 * kernel for every order, so that a multi-instance batch of instances of
 * different orders (pfd_batch_set_mode) merges their residuals into one
 * launch (not chosen by the autotuner).  pfd_create times
 * 0 and 1 and keeps the faster, then (refined contexts) the fused launch
 * against the separate residual and first pass.  The same sums in the same
 * order (results agree to rounding).  us[3] of pfd_get_residual_variant: us
 * per residual of 0 and 1, us per fused launch (0 if not timed).
 * Synchronises; drops captured graphs. */
pfd_status pfd_set_residual_variant(pfd_ctx* ctx, int variant);
pfd_status pfd_get_residual_variant(const pfd_ctx* ctx, int* variant, double* us);

/* Kernel configuration of the batched GEMMs per call site (0..3: the four
 * fast-diagonalisation passes, 4: the z transform; site -1: all).  cfg 0..7:
 * register tiles {TM, TN, SK} = {1,1,4} {2,2,1} {2,2,2} {3,3,1} {3,3,2}
 * {2,4,1} {4,2,1} {2,2,4}, a wave computing 16TM x 16TN of the output with SK
 * waves splitting the contraction; cfg 8..15: the shared small matrix staged in
 * LDS with the plane operand streamed, {W, SK} = {1,1} {2,1} {3,1} {1,2}
 * {2,2} {3,2} {1,4} {2,4} (W 16-wide tiles per wave along the small
 * dimension); cfg 16 (site 4 only, power-of-two 4 <= nz <= 256): the batched
 * FFT along z (two real node columns per complex transform, registers and one
 * LDS exchange) instead of the dense DFT matrices.  pfd_create times every
 * configuration that applies on the real
 * shapes and keeps each site's fastest (the autotuner); this overrides it (a
 * configuration that does not apply to a site falls back to cfg 0).
 * Synchronises; drops captured graphs. */
pfd_status pfd_set_gemm_config(pfd_ctx* ctx, int site, int cfg);
/* Chosen configuration per site (cfg[5]) and the autotuner's timings
 * (us[5*17]: site s, configuration k at us[17 s + k], microseconds per launch,
 * 0 where not tuned or not applicable; k = 16 is the FFT of site 4).  Either
 * may be NULL. */
pfd_status pfd_get_gemm_config(const pfd_ctx* ctx, int* cfg, double* us);

/* on != 0: pfd_step / pfd_step_async / pfd_march_to_equilibrium replay a
 * hipGraph of one whole step instead of launching its kernels one by one
 * (captured on first use on a stream the context owns, one graph per parity of
 * the time level and per step kind; the same kernels in the same order, so the
 * results are identical).  Graphs are bypassed while profiling is on.  on == 0
 * synchronises and frees the graphs. */
pfd_status pfd_set_graph(pfd_ctx* ctx, int on);

/* ------------------------------------------------------------------ batches
 * A batch steps independent contexts together: instances of uneven mesh,
 * order, parameters and precision (2D or 3D) that were all created on one
 * stream.  Each step is one hipGraph launch, made on first use per parity of
 * the time level and step kind, in one of two forms (pfd_batch_set_mode):
 *  PFD_BATCH_MULTI (default): multi-instance launches.  One step of every
 *    instance is recorded; the k-th launches of all instances that run the
 *    same kernel with the same work-group shape become one launch whose
 *    work-groups are the concatenation of the instances' grids (each
 *    instance keeps its own grid, arguments and buffers).  A step is as many
 *    launches as one instance's step times the number of distinct kernels at
 *    a position (e.g. one per element order for order-specialised kernels;
 *    residual variant 3 takes the order at run time), independent of the
 *    number of instances; results equal those of the instances stepped alone
 *    bit for bit.  The plan's tables and argument packs (about 4 bytes per
 *    work-group of a step, plus the arguments) are allocated when the
 *    graph is made.
 *  PFD_BATCH_BRANCHES: every instance's own launches as parallel graph
 *    branches (spread over nlanes capture streams, 1..16, default 4 when
 *    nlanes < 1).
 * The contexts stay owned by the caller, keep their own workspaces and
 * kernels, and are used as usual between batch steps (set/get fields,
 * sources, stats); destroy the batch before them.  Instances at different
 * time-level parities, or with profiling on, are stepped by plain launches in
 * order. */
typedef struct pfd_batch pfd_batch;
enum { PFD_BATCH_BRANCHES = 0, PFD_BATCH_MULTI = 1 };
pfd_status pfd_batch_create(pfd_ctx* const* ctxs, int n, int nlanes, pfd_batch** out);
/* Form of the batch's step graphs (PFD_BATCH_MULTI or PFD_BATCH_BRANCHES;
 * PFD_EINVAL otherwise).  A change drops the captured graphs (synchronises). */
pfd_status pfd_batch_set_mode(pfd_batch* b, int mode);
/* Launches per step of the multi-instance form (the largest captured plan);
 * -1 before the first capture. */
int pfd_batch_launches(const pfd_batch* b);
/* nsteps steps of every instance (equilibrium != 0: the equilibrium system),
 * then one synchronisation: PFD_ENONFINITE if any instance's state became
 * non-finite (that instance fails as in pfd_step; the others have stepped). */
pfd_status pfd_batch_step(pfd_batch* b, int nsteps, int equilibrium);
void pfd_batch_destroy(pfd_batch* b);
/* Message of the last error on b (or of the last failed pfd_batch_create when
 * b is NULL). */
const char* pfd_batch_last_error(const pfd_batch* b);

/* ------------------------------------------------------------ learned warm start
 * A small network, trained on equilibria the method computes, that maps the
 * three parameters of an equilibrium problem (voltage, permittivity ratio,
 * contact angle, each scaled to [-1, 1] by the caller) to the equilibrium
 * phase field on the field's grid (nz x ny x nx values, z slowest: the
 * context's field layout), used as the starting state of
 * pfd_march_to_equilibrium; the march to the residual tolerance still
 * decides the result.  Not in the paper.  A convolutional decoder:
 *   a1 = W1 p + b1, h1 = gelu(a1)   (64);  a2 = W2 h1 + b2, h2 = gelu(a2) (128)
 *   x0 = W3 h2 + b3                 (16 channels on a Z0 x Y0 x X0 latent grid,
 *                                    Z0 = ceil(nz / 8), likewise Y0, X0)
 *   for s = 1..3: a_s = conv(up(x_{s-1}); K_s) + c_s, x_s = gelu(a_s)
 *     (up doubles each axis by nearest neighbour; conv is 3x3x3, 16 -> 16
 *      channels, K_s[tap][out][in], tap = 9 (dz+1) + 3 (dy+1) + (dx+1); a
 *      neighbour outside the grid wraps along an axis that is periodic with
 *      8 Z0 = nz exactly, and is zero along any other)
 *   y = the nz x ny x nx corner of sum_c wo[c] x_3[c], plus bo
 *   loss = mean over batch and outputs of (y - t)^2
 * gelu(x) = x Phi(x).  FP32 master weights in one blob [W1 (64x3) | b1 |
 * W2 (128x64) | b2 | W3 (L0 x 128, L0 = 16 Z0 Y0 X0) | b3 | K1 (27x16x16) | c1
 * | K2 | c2 | K3 | c3 | wo (16) | bo (nz ny nx)], row-major, activations
 * channel-last.  The latent layer, the convolutions and all their backward
 * products run on the matrix cores with BF16 operands (rounded to nearest
 * even: h2, W3, x0, every x_s, the K_s, and dL/da_s, dL/dx0) and FP32
 * accumulation; Adam (0.9, 0.999, 1e-8).  Training inputs stay on the device:
 * params (S x 3, FP32) and targets (S x nz ny nx, FP32). */
typedef struct pfd_ws pfd_ws;
typedef struct {
  int hidden1;               /* must be 64  */
  int hidden2;               /* must be 128 */
  int channels;              /* must be 16  */
  int nz, ny, nx;            /* output grid, each 1..4096, nz ny nx >= 16 */
  int periodic_z, periodic_y, periodic_x;   /* nonzero: the axis may wrap */
  unsigned long long seed;   /* initial weights: N(0, 1/fan_in) (convolutions
                                N(0, 2/432)), wo N(0, 1e-4), biases 0 */
} pfd_ws_arch;
/* Weights in the blob, or 0 if the architecture is invalid. */
long pfd_ws_num_weights(const pfd_ws_arch* a);
pfd_status pfd_ws_workspace_query(const pfd_ws_arch* a, size_t* dev_bytes);
/* dev_ws: caller-owned device buffer of dev_bytes, 256-byte aligned. */
pfd_status pfd_ws_create(const pfd_ws_arch* a, void* dev_ws, size_t dev_bytes, void* stream, pfd_ws** out);
void pfd_ws_destroy(pfd_ws* ws);
const char* pfd_ws_last_error(const pfd_ws* ws);
/* Host copies of the FP32 weight blob (pfd_ws_num_weights floats). */
pfd_status pfd_ws_get_weights(pfd_ws* ws, float* host);
pfd_status pfd_ws_set_weights(pfd_ws* ws, const float* host);
/* bo = mean of the S training targets (device). */
pfd_status pfd_ws_init_output_bias(pfd_ws* ws, const float* targets, long S);
/* Gradient of the loss on the minibatch idx[0..B) (host indices into the
 * device params/targets, 1 <= B <= 32) into grad_host (a weight blob; may be
 * NULL) and *loss.  Synchronises. */
pfd_status pfd_ws_gradients(pfd_ws* ws, const float* params, const float* targets, const int* idx, int B,
                            float* grad_host, double* loss);
/* One Adam step with step size lr on the minibatch idx[0..B); *loss if not NULL. */
pfd_status pfd_ws_train_step(pfd_ws* ws, const float* params, const float* targets, const int* idx, int B,
                             float lr, double* loss);
/* steps Adam steps on minibatches of B drawn without replacement per epoch
 * from the S samples (shuffled by a generator seeded with seed), step size
 * decaying from lr to 0.05 lr (cosine); loss_history[steps] (host, may be
 * NULL) receives each step's minibatch loss.  Synchronises. */
pfd_status pfd_ws_train(pfd_ws* ws, const float* params, const float* targets, long S, int steps, int B, float lr,
                        unsigned long long seed, double* loss_history);
/* Prediction for one input p_host[3] into out (device, nz ny nx FP64).  With
 * weights (device, nz ny nx FP64: the quadrature weights of the field's integral)
 * the prediction is shifted by a constant so that sum(weights * out) = mass
 * (mass conservation of eq. 16 fixes the equilibrium's integral).  Synchronises. */
pfd_status pfd_ws_predict(pfd_ws* ws, const float* p_host, const double* weights, double mass, double* out);

/* Mass and energy of the current state (see pfd_stats) for every instance:
 * out holds nbatch entries in 2D, one in 3D (host memory).  Uses E from the
 * last step or pfd_init_potential.  Stream-ordered, then synchronises. */
pfd_status pfd_get_stats(pfd_ctx* ctx, pfd_stats* out);

/* March the equilibrium system (eq. 16 with u = 0: potential, psi and phi
 * stages only) until r_m = max |phi^{m+1} - phi^m| over every node and
 * instance is <= tol, checked after each step, or max_steps steps.  *steps
 * (may be NULL) receives the steps taken, *residual (may be NULL) the last
 * r_m.  PFD_ENOCONV if max_steps is reached, PFD_ENONFINITE (and the context
 * fails) on a non-finite state.  Synchronises once per step. */
pfd_status pfd_march_to_equilibrium(pfd_ctx* ctx, double tol, long max_steps, long* steps,
                                    double* residual);

/* Copy a field in or out.  level 0 = time level n, -1 = level n-1 (u, P, phi,
 * V, psi have two levels; E only level 0).  src/dst hold planes*Ny*Nx doubles,
 * on the device when on_device != 0 (stream-ordered, no sync) else on the
 * host (synchronous).  Setting level 0 of u, P, phi or V without setting
 * level -1 afterwards also copies it to level -1 (BDF start, Sec. 3.1). */
pfd_status pfd_set_field(pfd_ctx* ctx, int field, int level, const double* src, int on_device);
pfd_status pfd_get_field(pfd_ctx* ctx, int field, int level, double* dst, int on_device);

/* Set one source array (see pfd_source); NULL resets it to zero. */
pfd_status pfd_set_source(pfd_ctx* ctx, int source, const double* src, int on_device);

/* Initial potential by the fixed point of Remark 3.1: iterate eq. (54)/(74)
 * with phi* = phi^0 and V* = previous iterate until
 * max|dV| <= tol * max(1, max|V|) or max_iter iterations.  Stores the result
 * at levels n and n-1 of V and updates E.  Synchronises.  PFD_ENOCONV if the
 * tolerance is not met. */
pfd_status pfd_init_potential(pfd_ctx* ctx, double tol, int max_iter, int* iters);

/* Advance nsteps time steps (Algorithm 1 or 2).  equilibrium != 0 runs the
 * simpler system of Sec. 2.4 (eqs. 15c-d and 16: V, E, psi, phi with u = 0)
 * instead of the full step.  Sources are held fixed over the nsteps steps.
 * Stream-ordered; synchronises once at the end to read the status word.
 * Returns PFD_ENONFINITE if a non-finite value appeared. */
pfd_status pfd_step(pfd_ctx* ctx, int nsteps, int equilibrium);

/* Same as pfd_step without the final synchronisation or status read: for
 * timing loops and graph capture.  Check pfd_get_diag afterwards. */
pfd_status pfd_step_async(pfd_ctx* ctx, int nsteps, int equilibrium);

/* Solve (K + (c_f + beta_p^2) M) x = b for solve family fam on every plane (in 3D the
 * planes are the packed spectral planes: 0 = Re k=0, 1 = Re k=Nz/2, 2k / 2k+1 = Re / Im of
 * mode k, beta_p = 2 pi k / Lz),
 * with x = x_in on the family's Dirichlet nodes (eqs. 54-59 operators).  b and
 * x are device arrays of planes*Ny*Nx doubles; x holds the initial guess and
 * the Dirichlet values on entry and the solution on exit.  For a singular
 * family (no Dirichlet node and zero shift) b is projected onto the range and
 * the solution has int_h x = 0.  Uses the context's precision setting. */
pfd_status pfd_solve(pfd_ctx* ctx, int fam, const double* b, double* x);

/* y = (K + (c_f + beta_p^2) M) x on every plane (device arrays). */
pfd_status pfd_apply(pfd_ctx* ctx, int fam, const double* x, double* y);

/* pfd_solve for callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same kernels in the same order (the
 * result equals pfd_solve's), with the solve's scratch (residual, fast-diagonalisation
 * intermediates, refinement test sums and gate, electrode gap buffers) taken from one static
 * device array of 64 MiB that the library holds on every device until the process ends,
 * instead of the context's workspace.  Allocates nothing.  The context's device must be
 * current.  PFD_ENOMEM (message with the bytes needed) when the context's planes * Nx * Ny
 * exceeds what the array holds (about 10 doubles per node: 838,000 nodes).  Every call on a
 * device shares the array: calls that overlap on one device race; serialise them. */
pfd_status pfd_solve_static(pfd_ctx* ctx, int fam, const double* b, double* x);

/* Kernel classes timed by pfd_profile_read */
enum {
  PFD_PROF_GEMM64 = 0,   /* fast-diagonalisation GEMM passes, FP64 (MFMA)          */
  PFD_PROF_GEMM32 = 1,   /* fast-diagonalisation GEMM passes, FP32 (MFMA)          */
  PFD_PROF_RESID = 2,    /* FP64 residual r = b - A x                               */
  PFD_PROF_ELEM = 3,     /* element kernels (sum-factorised terms, weak forms)     */
  PFD_PROF_NODAL = 4,    /* nodal kernels (direct-stiffness sums, right sides)      */
  PFD_PROF_OTHER = 5,    /* reductions, guards                                      */
  PFD_PROF_ZFFT = 6,     /* z transforms (packed real DFT GEMMs, 3D)                */
  PFD_PROF_NCLASS = 7
};

/* Enable (on != 0) or disable per-launch timing: when enabled, every kernel launch of
 * the context is bracketed by two HIP events on the context's stream (this adds a
 * little host overhead per launch; time the step loop with profiling off).  Enabling
 * clears earlier records. */
pfd_status pfd_profile_enable(pfd_ctx* ctx, int on);

/* Total device time (ms) and number of launches of one kernel class since profiling
 * was enabled.  Synchronises the stream. */
pfd_status pfd_profile_read(pfd_ctx* ctx, int cls, double* total_ms, long* launches);

/* Average device time (microseconds) of one launch of a kernel class, measured by
 * replaying it reps times back to back on the context's own shapes, buffers and
 * stream between two HIP events (GEMM classes: the four fast-diagonalisation passes
 * of one velocity correction; PFD_PROF_RESID: the velocity residual).  Writes only
 * scratch buffers; the state is unchanged.  Synchronises. */
pfd_status pfd_profile_replay(pfd_ctx* ctx, int cls, int reps, double* avg_us);

#ifdef __cplusplus
}
#endif
#endif /* PFD_H */
