// lbm_macros_noalloc: the moments and FP64 sums of lbm_macros without any
// allocation, for callers that cannot allocate (HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).  The block partial sums go to a
// file-scope device array instead of library-allocated memory; its address on
// each device is looked up once (lbm_init_domain calls noalloc_setup with the
// domain's device current) and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lbm.h"
#include "error.hpp"
#include "internal.hpp"

namespace lbm {
namespace {

constexpr int NOALLOC_BLOCKS = 1024;                 // workgroups of the persistent macros kernel
constexpr int NOALLOC_DOUBLES = NOALLOC_BLOCKS * NPART;

// Partial sums of the no-allocation moments call (64 KiB; one copy per device,
// held until the process ends).  Host code must use its per-device address from
// hipGetSymbolAddress, never this name.
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};

}  // namespace

// Look up the scratch array's address on the current device (once per device).
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void* p = nullptr;
    g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_err[device] == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

}  // namespace lbm

using namespace lbm;

extern "C" int lbm_macros_noalloc(lbm_domain d, double* rho, double* u, double* sums) {
  if (!d || !sums) return set_error(LBM_EINVAL, "null argument");
  if (d->device < 0 || d->device >= MAX_DEVICES) return set_error(LBM_EDEVICE, "domain without a device");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[d->device] || g_ptr[d->device] == nullptr)
      return set_error(LBM_EDEVICE, std::string("no scratch address on device ") + std::to_string(d->device) + ": " +
                                        (g_done[d->device] ? hipGetErrorString(g_err[d->device]) : "not set up"));
    ptr = g_ptr[d->device];
  }
  // the persistent grid: at most NOALLOC_BLOCKS workgroups walk the lattice's blocks
  const int64_t grid = d->red_blocks < NOALLOC_BLOCKS ? d->red_blocks : NOALLOC_BLOCKS;
  if (grid * NPART > NOALLOC_DOUBLES) return set_error(LBM_EINVAL, "partial sums exceed the scratch array");
  MacroParams p{};
  p.g = d->g;
  p.src = d->buf[d->cur];
  p.lk.seg_fluid = d->seg_fluid;
  p.lk.seg_fbase = d->seg_fbase;
  p.lk.row_src = d->row_src;
  p.lk.seg_bnd = d->seg_bnd;
  p.lk.seg_lbase = d->seg_lbase;
  p.lk.lld = d->lld;
  p.lk.lnode = d->lnode;
  p.lk.lq = d->lq;
  p.lk.lg = d->lg;
  p.lk.lv_in = d->lv[d->cur];
  p.lk.luv = d->luv;
  for (int a = 0; a < 3; ++a) p.force[a] = d->desc.force[a];
  p.rho = rho;
  p.u = u;
  p.uprev = nullptr;                       // no residual: its previous field would need N * D doubles
  p.partials = static_cast<double*>(ptr);  // every row is written by its workgroup: nothing to clear
  p.nblocks = d->red_blocks;
  hipError_t e = launch_macros(d->desc.lattice, d->desc.storage, p, grid, d->stream);
  if (e == hipSuccess) e = launch_reduce(static_cast<const double*>(ptr), grid, sums, d->stream);
  if (e != hipSuccess) return set_error(LBM_EDEVICE, std::string("macros: ") + hipGetErrorString(e));
  clear_error();
  return LBM_OK;
}
