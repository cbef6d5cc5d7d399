// ndtm_apply without device allocation: the variant of ndtm_apply (FP64) for
// callers that cannot allocate (code under graph capture, tight serving loops).
//
// Its four internal half fields live in `scratch`, a fixed device array of this
// file.  In host code `scratch` only names the symbol, so the array's device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) when a context is created, and every launch takes that address.  The
// array is shared by every call on a device and keeps the last call's contents;
// calls that overlap on one GPU (other streams, other threads) race on it.
#include <mutex>

#include "ctx.h"

namespace ndtm {

constexpr size_t kScratchBytes = (size_t)128 << 20;  // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};
static hipError_t g_scratch_err[kMaxDevices] = {};
static bool g_scratch_done[kMaxDevices] = {};

// Called by ndtm_create with `device` current: resolves this device's copy of scratch.
void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
  g_scratch_done[device] = true;
}

static void* scratch_of(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices || !g_scratch_done[device]) {
    *err = hipErrorNotInitialized;
    return nullptr;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

size_t ndtm_apply_noalloc_max_bytes(void) { return kScratchBytes; }

int ndtm_apply_noalloc(ndtm_ctx* c, int op, void* y_dev, const void* x_dev, double param, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!y_dev || !x_dev || y_dev == x_dev) return fail(c, NDTM_EINVAL, "apply_noalloc: null or aliased pointers");
  if (op < NDTM_OP_QHAT || op > NDTM_OP_HOP_OE) return fail(c, NDTM_EINVAL, "apply_noalloc: unknown operator");
  if (!c->have_gauge || !c->have_params)
    return fail(c, NDTM_ESTATE, "apply_noalloc: set_gauge and set_params first");
  const size_t n = half_elems(c);
  const size_t need = 4 * n * sizeof(double2);
  if (need > kScratchBytes)
    return fail(c, NDTM_EINVAL,
                "apply_noalloc: the lattice needs " + std::to_string(need) + " bytes of scratch (4 FP64 half fields), "
                "more than the fixed " + std::to_string(kScratchBytes) + "; use ndtm_apply");
  NDTM_HIP(c, hipSetDevice(c->device));
  hipError_t e = hipSuccess;
  double2* base = static_cast<double2*>(scratch_of(c->device, &e));
  if (!base) return hip_check(c, e == hipSuccess ? hipErrorInvalidSymbol : e, "apply_noalloc: scratch address");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HalfField F[4];
  for (int i = 0; i < 4; ++i) {
    F[i].prec = P64;
    F[i].v = base + (size_t)i * n;
  }
  const HalfField &X = F[0], &Y = F[1], &T = F[2], &W = F[3];
  const double2* x = static_cast<const double2*>(x_dev);
  double2* y = static_cast<double2*>(y_dev);
  switch (op) {
    case NDTM_OP_QHAT:
      launch_pack_half(c->g, x, X, st);
      apply_qhat(c, P64, Y, X, T, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_QHAT2:
      launch_pack_half(c->g, x, X, st);
      apply_qhat2(c, P64, Y, X, W, T, param, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_SHAT_SHIFT:
      launch_pack_half(c->g, x, X, st);
      apply_sshift(c, P64, Y, X, T, param, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_DFULL:
      launch_pack_full(c->g, x, T, X, st);
      apply_dfull(c, P64, W, Y, T, X, param, st);
      launch_unpack_full(c->g, W, Y, y, st);
      break;
    case NDTM_OP_HOP_EO:
      launch_pack_half(c->g, x, X, st);
      hop(c, P64, EPI_PLAIN, RED_NONE, 0, X, Y, nullptr, nullptr, 0, 0, 0, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    default:  // NDTM_OP_HOP_OE
      launch_pack_half(c->g, x, X, st);
      hop(c, P64, EPI_PLAIN, RED_NONE, 1, X, Y, nullptr, nullptr, 0, 0, 0, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
  }
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

}  // extern "C"
