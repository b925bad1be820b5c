// pfd_solve_static: the constant-matrix solve of pfd_solve for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses that forbid
// allocation).  Its scratch -- the FP64 residual, the fast-diagonalisation intermediates, the
// refinement test's partial sums and gate, the singular-plane sums and the electrode gap
// buffers -- comes from one file-scope device array instead of the context's workspace.
// The array holds PFD_STATIC_SCRATCH_BYTES on every device the library is loaded on, until
// the process ends; every call on a device shares it, so calls that overlap on one device
// race (serialise them, e.g. on one stream).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "pfd_internal.h"

#define PFD_STATIC_SCRATCH_BYTES (64L << 20)
#define PFD_STATIC_MAX_DEVICES 64

static __device__ __align__(256) double scratch[PFD_STATIC_SCRATCH_BYTES / sizeof(double)];

namespace {

std::mutex g_mu;
double* g_ptr[PFD_STATIC_MAX_DEVICES] = {};

// Device address of this device's copy of the array, looked up once per device (the array's
// name in host code is only a stand-in for the symbol, never a device address).
hipError_t scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    double* p = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" pfd_status pfd_solve_static(pfd_ctx* c, int fam, const double* b, double* x) {
  if (!c || !b || !x || fam < 0 || fam > 4) return PFD_EINVAL;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { c->err = hipGetErrorString(e); return PFD_EHIP; }
  if (dev != c->device) {
    c->err = "pfd_solve_static: make the context's device current first";
    return PFD_EINVAL;
  }
  if (dev < 0 || dev >= PFD_STATIC_MAX_DEVICES) { c->err = "pfd_solve_static: device index too large"; return PFD_EINVAL; }
  // carve the slices the solve uses (the context's own capacities), 256-byte aligned
  const long tot = (long)c->planes * c->Ng;
  const long ng = c->elec.ng;
  const long sizes[8] = {3 * tot, 3 * tot, 3 * tot, tot, 2 * c->rpart_max, 32, 32L * c->planes, c->planes * ng + 1};
  long need = 0;
  long off[8];
  for (int i = 0; i < 8; ++i) {
    off[i] = need;
    need += (sizes[i] + 31) & ~31L;   // doubles, rounded to 256 bytes
  }
  if (need * (long)sizeof(double) > PFD_STATIC_SCRATCH_BYTES) {
    c->err = "pfd_solve_static: the solve needs " + std::to_string(need * sizeof(double)) +
             " bytes of scratch, more than the " + std::to_string(PFD_STATIC_SCRATCH_BYTES) +
             " bytes of the static array (use pfd_solve)";
    return PFD_ENOMEM;
  }
  double* base = nullptr;
  e = scratch_ptr(dev, &base);
  if (e != hipSuccess) { c->err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e); return PFD_EHIP; }
  // the context's scratch pointers are pointed at the slices for this call only
  double *r = c->r, *tmp = c->tmp, *tmp2 = c->tmp2, *ybuf = c->Ybuf, *rpart = c->d_rpart, *part = c->d_part;
  double* dG = c->elec.d_dG;
  int* gate = c->d_gate;
  const int prof = c->prof_on;
  c->r = base + off[0];
  c->tmp = base + off[1];
  c->tmp2 = base + off[2];
  c->Ybuf = base + off[3];
  c->d_rpart = base + off[4];
  c->d_gate = reinterpret_cast<int*>(base + off[5]);
  c->d_part = base + off[6];
  if (ng > 0) c->elec.d_dG = base + off[7];
  c->prof_on = 0;   // no timing events (they are created on demand)
  e = pfd::solve(c, fam, b, x, 1, 1, nullptr, false);
  c->r = r;
  c->tmp = tmp;
  c->tmp2 = tmp2;
  c->Ybuf = ybuf;
  c->d_rpart = rpart;
  c->d_gate = gate;
  c->d_part = part;
  c->elec.d_dG = dG;
  c->prof_on = prof;
  if (e != hipSuccess) { c->err = hipGetErrorString(e); return PFD_EHIP; }
  return PFD_OK;
}
