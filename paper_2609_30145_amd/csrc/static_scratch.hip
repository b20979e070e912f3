// Allocation-free forward + logL: sps_logl with the per-call scratch of the forward path
// (batch keys, weight rows, K-tile occupancy bits, per-point rows, the attenuated
// rest-frame spectrum, line luminosities, the tile list, the nebular-continuum masses)
// carved from one file-scope device array
// instead of the observation's workspace.  For callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops, harnesses that forbid it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sps.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

namespace sps {

constexpr size_t kStaticScratchBytes = (size_t)SPS_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  Host code never passes this name to
// a kernel or a copy: it is a host-side stand-in; the device address of each GPU's copy
// comes from hipGetSymbolAddress (static_scratch_init) and is kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices] = {};

// Looks up the device address of `scratch` on `device` (once per device), with that device
// current; restores the calling thread's current device.
sps_status static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(SPS_E_INVAL, "device %d outside [0, %d)", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return SPS_OK;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return fail(SPS_E_HIP, "hipGetDevice failed");
  if (prev != device && hipSetDevice(device) != hipSuccess) return fail(SPS_E_HIP, "hipSetDevice(%d) failed", device);
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (prev != device) (void)hipSetDevice(prev);
  if (e != hipSuccess || !ptr)
    return fail(SPS_E_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
  g_scratch[device] = ptr;
  return SPS_OK;
}

static void *static_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Bytes of scratch the forward path needs for B points at a precision (the same buffers
// as Workspace::create holds for the forward pass, at their per-precision sizes).
size_t static_scratch_bytes(const DevLib &g, int B, int prec) {
  const size_t Bp = (size_t)(B + kMAlign - 1) / kMAlign * kMAlign;
  const int mask_words = (g.K_pad / kKTile + 31) / 32;
  const size_t w_el = prec == SPS_FP64 ? 8 : 4;   // 16-bit paths: hi and residual planes
  const size_t f_el = prec == SPS_FP64 ? 8 : 4;
  return align256(Bp * 8) + align256(Bp * 4) + align256(Bp * g.K_pad * w_el) + align256(Bp * mask_words * 4) +
         align256(Bp * sizeof(PointRow)) + align256(Bp * g.N_pad * f_el) +
         align256(Bp * (size_t)(g.n_line > 0 ? g.n_line : 1) * 8) + align256(tile_list_ints(Bp, g.N_pad) * 4) +
         align256(Bp * (size_t)(g.has_cont ? g.neb_a1 - g.neb_a0 : 1) * 8);
}

}  // namespace sps

using namespace sps;

extern "C" sps_status sps_logl_static(const sps_library *L, const sps_obs *o, const double *theta, int32_t B,
                                      int32_t prec, double *logl, double *model, void *stream) {
  if (!L || !o || !theta || !logl) return fail(SPS_E_INVAL, "sps_logl_static: NULL argument");
  if (o->lib != L) return fail(SPS_E_INVAL, "observation belongs to another library");
  if (L->device < 0) return fail(SPS_E_STATE, "host-only library");
  if (B < 1) return fail(SPS_E_SHAPE, "B=%d must be >= 1", B);
  if (!precision_built(L, prec)) return fail(SPS_E_INVAL, "precision %d not built into this library", prec);
  if (o->host.calib_mode != SPS_CALIB_NONE || o->host.lm_mode != SPS_LINEMARG_NONE)
    return fail(SPS_E_INVAL, "sps_logl_static: a calibration polynomial or line marginalisation needs the "
                "observation's own workspace (sps_logl)");
  const DevLib &g = L->dev;
  const size_t need = static_scratch_bytes(g, B, prec);
  if (need > kStaticScratchBytes)
    return fail(SPS_E_SHAPE, "sps_logl_static: B=%d at precision %d needs %zu bytes of scratch, more than the %zu "
                "of the static array (use sps_logl)", B, prec, need, kStaticScratchBytes);
  unsigned char *base = (unsigned char *)static_scratch_ptr(L->device);
  if (!base) return fail(SPS_E_STATE, "static scratch not set up on device %d", L->device);
  // a workspace view of the scratch (it owns nothing: its allocation list stays empty)
  Workspace w;
  w.max_batch = B;
  w.B_pad_max = (B + kMAlign - 1) / kMAlign * kMAlign;
  w.mask_words = (g.K_pad / kKTile + 31) / 32;
  const size_t Bp = w.B_pad_max;
  const size_t w_el = prec == SPS_FP64 ? 8 : 4, f_el = prec == SPS_FP64 ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t n) {
    void *p = base + off;
    off += align256(n);
    return p;
  };
  w.keys = (double *)take(Bp * 8);
  w.ranks = (int *)take(Bp * 4);
  w.W = take(Bp * g.K_pad * w_el);
  w.rowmask = (uint32_t *)take(Bp * w.mask_words * 4);
  w.rows = (PointRow *)take(Bp * sizeof(PointRow));
  w.F = take(Bp * g.N_pad * f_el);
  w.Lline = (double *)take(Bp * (size_t)(g.n_line > 0 ? g.n_line : 1) * 8);
  w.tiles = (int *)take(tile_list_ints(Bp, g.N_pad) * 4);
  w.WQ = (double *)take(Bp * (size_t)(g.has_cont ? g.neb_a1 - g.neb_a0 : 1) * 8);
  w.counter = nullptr;
  return launch_forward(L, w, o->dev_obs, nullptr, theta, B, prec, logl, model, o->host.n_data, false,
                        o->host.n_data, &o->host, nullptr, (hipStream_t)stream);
}
