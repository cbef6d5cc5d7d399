// C-ABI entry points (context, gauge field, parameters, operator application,
// profiling) and the internal operator helpers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "ctx.h"

namespace ndtm {

int fail(ndtm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_check(ndtm_ctx* c, hipError_t e, const char* what) {
  return fail(c, NDTM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void* ws_get(ndtm_ctx* c, const std::string& name, size_t bytes) {
  DevBuf& b = c->bufs[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) dev_free(c, b.p);
  b.p = dev_alloc(c, bytes);
  b.bytes = 0;
  if (!b.p) {
    c->bufs.erase(name);
    return nullptr;
  }
  (void)hipMemset(b.p, 0, bytes);
  b.bytes = bytes;
  return b.p;
}

size_t ws_bytes(const ndtm_ctx* c, const std::string& name) {
  auto it = c->bufs.find(name);
  return it == c->bufs.end() ? 0 : it->second.bytes;
}

void ws_free_prefix(ndtm_ctx* c, const std::string& prefix) {
  for (auto it = c->bufs.begin(); it != c->bufs.end();) {
    if (it->first.compare(0, prefix.size(), prefix) == 0) {
      dev_free(c, it->second.p);
      it = c->bufs.erase(it);
    } else {
      ++it;
    }
  }
}

size_t half_elems(const ndtm_ctx* c) { return (size_t)24 * c->g.stride; }

HalfField half_field(ndtm_ctx* c, const std::string& name, int prec) {
  HalfField f;
  f.prec = prec;
  const size_t n = half_elems(c);
  const size_t esz = prec == P64 ? 16 : (prec == P32 ? 8 : 4);
  f.v = ws_get(c, name + (prec == P64 ? "#64" : prec == P32 ? "#32" : "#16"), n * esz);
  if (prec == P16) f.sc = static_cast<float*>(ws_get(c, name + "#sc", (size_t)c->g.stride * 4));
  return f;
}

// Moves the timed launches that have completed (in launch order per class) into the
// class totals and their event pairs back to the free list.
static void harvest_events(ndtm_ctx* c) {
  for (int k = 0; k < NDTM_PROF_NCLASS; ++k) {
    auto& used = c->ev_used[k];
    size_t done = 0;
    for (; done < used.size(); ++done) {
      if (hipEventQuery(used[done].second) != hipSuccess) break;
      float ms = 0;
      if (hipEventElapsedTime(&ms, used[done].first, used[done].second) != hipSuccess) break;
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
      c->ev_free.push_back(used[done]);
    }
    used.erase(used.begin(), used.begin() + done);
  }
}

static std::pair<hipEvent_t, hipEvent_t> take_events(ndtm_ctx* c) {
  // creating events costs far more than recording them: recycle completed pairs first
  if (c->ev_free.empty()) harvest_events(c);
  if (!c->ev_free.empty()) {
    auto e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  std::pair<hipEvent_t, hipEvent_t> e;
  (void)hipEventCreate(&e.first);
  (void)hipEventCreate(&e.second);
  return e;
}

ProfScope::ProfScope(ndtm_ctx* c_, int cls_, double bytes, hipStream_t st_, double moved)
    : c(c_), cls(cls_), st(st_) {
  if (!((c->prof_mask >> cls) & 1)) return;
  ev = take_events(c);
  (void)hipEventRecord(ev.first, st);
  c->prof_bytes[cls] += bytes;
  c->prof_moved[cls] += moved >= 0 ? moved : bytes;
}

ProfScope::~ProfScope() {
  if (!((c->prof_mask >> cls) & 1)) return;
  (void)hipEventRecord(ev.second, st);
  c->ev_used[cls].push_back(ev);
}

// Algorithmic bytes per output site of one stencil pass: 8 links of 18 reals and one
// input and one output doublet spinor, each read or written once.  The fused site
// epilogues also read one or two site vectors; those bytes count as moved, not as
// the pass's algorithmic bytes.
// strict bytes per output site (8 links with two rows, the input and output spinors) and
// per extra epilogue vector; P32H: FP16 links with FP32 fields
static const double kHopBase[4] = {1920.0, 960.0, 488.0, 672.0}, kHopVec[4] = {384.0, 192.0, 100.0, 192.0};
static double hop_epi_vectors(int epi) {
  if (epi == EPI_QHAT || epi == EPI_SITE || epi == EPI_SITE_Q) return 1;
  if (epi == EPI_QHAT_SIG) return 2;
  return 0;
}

// smallest |U01|^2 + |U02|^2 of every link for the eight-parameter form: the rebuild
// divides by it (its numerators are of the same order, so the rebuilt entries keep FP64
// accuracy down to tiny norms; the bound only keeps out links whose first row is
// (u, 0, 0) to within rounding, such as unit links)
constexpr double kR8MinNorm = 1e-20;

void hop(ndtm_ctx* c, int prec, int epi, int red, int parity, const HalfField& in, const HalfField& out,
         const HalfField* xs, const HalfField* zs, double ms, double hop_coef, double sigma,
         double* partials, hipStream_t st) {
  // the FP32-field stencil on FP16 links times into the FP32 class
  const int cls = prec == P32H ? P32 : prec, lp = prec == P32H ? P16 : prec;
  ProfScope ps(c, NDTM_PROF_HOP_F64 + cls, kHopBase[prec] * c->g.vh, st,
               (kHopBase[prec] + hop_epi_vectors(epi) * kHopVec[prec]) * c->g.vh);
  OpParams op = c->op;
  op.skip = c->hop_skip;
  launch_hop(prec, epi, red, c->g, parity, op, c->U[lp][parity], c->U[lp][1 - parity], in, out,
             xs, zs, ms, hop_coef, sigma, partials, st);
}

void apply_qhat(ndtm_ctx* c, int prec, const HalfField& y, const HalfField& x, const HalfField& tmp_e,
                hipStream_t st) {
  hop(c, prec, EPI_AINV, RED_NONE, 0, x, tmp_e, nullptr, nullptr, 0, 0, 0, nullptr, st);
  hop(c, prec, EPI_QHAT, RED_NONE, 1, tmp_e, y, &x, nullptr, 0, 0, 0, nullptr, st);
}

void apply_qhat2(ndtm_ctx* c, int prec, const HalfField& w, const HalfField& p, const HalfField& u,
                 const HalfField& tmp_e, double sigma, double* partials, hipStream_t st) {
  apply_qhat(c, prec, u, p, tmp_e, st);
  hop(c, prec, EPI_AINV, RED_NONE, 0, u, tmp_e, nullptr, nullptr, 0, 0, 0, nullptr, st);
  hop(c, prec, EPI_QHAT_SIG, partials ? RED_REDOT : RED_NONE, 1, tmp_e, w, &u, &p, 0, 0, sigma, partials,
      st);
}

void apply_sshift(ndtm_ctx* c, int prec, const HalfField& y, const HalfField& x, const HalfField& tmp_e,
                  double m, hipStream_t st) {
  hop(c, prec, EPI_AINV, RED_NONE, 0, x, tmp_e, nullptr, nullptr, 0, 0, 0, nullptr, st);
  hop(c, prec, EPI_SITE, RED_NONE, 1, tmp_e, y, &x, nullptr, m, -0.25, 0, nullptr, st);
}

void apply_dfull(ndtm_ctx* c, int prec, const HalfField& ye, const HalfField& yo, const HalfField& xe,
                 const HalfField& xo, double m, hipStream_t st) {
  hop(c, prec, EPI_SITE, RED_NONE, 0, xo, ye, &xe, nullptr, 0.0, -0.5, 0, nullptr, st);
  hop(c, prec, EPI_SITE, RED_NONE, 1, xe, yo, &xo, nullptr, m, -0.5, 0, nullptr, st);
}

double norm2_host(ndtm_ctx* c, const double2* x, size_t n, hipStream_t st) {
  const int g = blas_norm2_partials(x, n, c->partials, st);
  blas_finalize(c->partials, g, 1, c->dscal, st);
  (void)hipMemcpyAsync(c->hscal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  return c->hscal[0];
}

double2 dot_host(ndtm_ctx* c, const double2* x, const double2* y, size_t n, hipStream_t st) {
  const int g = blas_dot_partials(x, y, n, c->partials, st);
  blas_finalize(c->partials, g, 2, c->dscal, st);
  (void)hipMemcpyAsync(c->hscal, c->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  return make_double2(c->hscal[0], c->hscal[1]);
}

int clover_build(ndtm_ctx* c, hipStream_t st) {
  if (c->csw == 0.0) {
    c->op.clover = 0;
    return NDTM_OK;
  }
  if (!c->have_gauge || !c->have_params) return NDTM_OK;  // built once both are set
  const size_t sm = (size_t)72 * c->g.stride, si = (size_t)144 * c->g.stride;
  for (int q = 0; q < 2; ++q) {
    const size_t es = q == 0 ? 8 : 4;
    for (int par = 0; par < 2; ++par)
      if (!c->clv_m[q][par] && !(c->clv_m[q][par] = dev_alloc(c, sm * es)))
        return fail(c, NDTM_ENOMEM, "clover: site blocks");
    if (!c->clv_inv[q] && !(c->clv_inv[q] = dev_alloc(c, si * es))) return fail(c, NDTM_ENOMEM, "clover: site blocks");
  }
  if (!c->clv_bad && !(c->clv_bad = static_cast<unsigned*>(dev_alloc(c, 256))))
    return fail(c, NDTM_ENOMEM, "clover: counter");
  unsigned bad[2] = {0, 0};
  for (int par = 0; par < 2; ++par) {
    launch_clover_build(c->g, (const double2*)c->U[P64][0], (const double2*)c->U[P64][1], par, c->op.a, c->csw,
                        c->mubar, c->epsbar, (double*)c->clv_m[0][par], par == 0 ? (double*)c->clv_inv[0] : nullptr,
                        c->clv_bad, st);
    NDTM_HIP(c, hipMemcpyAsync(&bad[par], c->clv_bad, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    NDTM_HIP(c, hipStreamSynchronize(st));
    launch_to_f32((const double*)c->clv_m[0][par], (float*)c->clv_m[1][par], (long)sm, st);
  }
  launch_to_f32((const double*)c->clv_inv[0], (float*)c->clv_inv[1], (long)si, st);
  NDTM_HIP(c, hipGetLastError());
  NDTM_HIP(c, hipStreamSynchronize(st));
  if (bad[0] + bad[1]) {
    c->op.clover = 0;
    return fail(c, NDTM_EINVAL, "clover: M^2 + mubar^2 - epsbar^2 is singular on " + std::to_string(bad[0] + bad[1]) +
                                    " site blocks");
  }
  for (int q = 0; q < 2; ++q) {
    for (int par = 0; par < 2; ++par) c->op.clv_m[q][par] = c->clv_m[q][par];
    c->op.clv_inv[q] = c->clv_inv[q];
  }
  c->op.clover = 1;
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

int ndtm_set_clover(ndtm_ctx* c, double csw) {
  if (!c) return NDTM_EINVAL;
  if (!std::isfinite(csw)) return fail(c, NDTM_EINVAL, "set_clover: c_sw must be finite");
  NDTM_HIP(c, hipSetDevice(c->device));
  c->csw = csw;
  ndtm_mg_free(c);
  return clover_build(c, nullptr);
}

int ndtm_create(const int dims[4], int bc_flags, int device, ndtm_ctx** out) {
  if (!dims || !out) return NDTM_EINVAL;
  *out = nullptr;
  long long V = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2 || (dims[i] & 1)) return NDTM_EINVAL;
    V *= dims[i];
  }
  // the stencil addresses a field through 32-bit byte offsets from each
  // component array: 13 x (V/2 + 512) x 16 bytes must stay below 4 GiB
  if (13.0 * (double)(V / 2 + 512) * 16.0 >= 4294967296.0) return NDTM_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NDTM_EHIP;
  if (hipSetDevice(device) != hipSuccess) return NDTM_EHIP;
  noalloc_setup(device);
  ndtm_ctx* c = new (std::nothrow) ndtm_ctx();
  if (!c) return NDTM_ENOMEM;
  c->device = device;
  c->V = V;
  c->g.T = dims[0];
  c->g.Lz = dims[1];
  c->g.Ly = dims[2];
  c->g.Lx = dims[3];
  c->g.vh = (int)(V / 2);
  // one extra 256-element block keeps the 24 component arrays (and the 36 link
  // arrays) of a field off power-of-two spacings, which alias in the HBM channels
  c->g.stride = (int)((V / 2 + 255) / 256 * 256) + 256;
  c->g.antiperiodic = bc_flags & 1;
  c->partials_n = (size_t)hop_grid(c->g) * 4 + 4096 * 80;
  if (hipMalloc(&c->partials, c->partials_n * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->dscal, kScalN * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->mms_S, MS_SIZE * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->mms_H, (size_t)kMaxDefer * kMaxShifts * kHistStride * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->mms_L, (size_t)kLanczosIters * kMaxShifts * kHistStride * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->mms_C, (size_t)kMaxShifts * kCoefStride * sizeof(double)) != hipSuccess ||

      hipMalloc(&c->vred, kVredN * sizeof(double)) != hipSuccess || hipMemset(c->vred, 0, kVredN * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&c->hscal, kScalN * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    ndtm_destroy(c);
    return NDTM_ENOMEM;
  }
  *out = c;
  return NDTM_OK;
}

void ndtm_mg_free(ndtm_ctx* c);
void ndtm_mlp_free(ndtm_ctx* c);

void ndtm_destroy(ndtm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  ndtm_mg_free(c);
  ndtm_mlp_free(c);
  for (auto& kv : c->bufs) dev_free(c, kv.second.p);
  c->bufs.clear();
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 2; ++q) dev_free(c, c->U[p][q]);
  for (int q = 0; q < 2; ++q) dev_free(c, c->U8[q]);
  for (int q = 0; q < 2; ++q) {
    dev_free(c, c->clv_m[q][0]);
    dev_free(c, c->clv_m[q][1]);
    dev_free(c, c->clv_inv[q]);
  }
  dev_free(c, c->clv_bad);
  arena_release(c);
  if (c->partials) (void)hipFree(c->partials);
  if (c->dscal) (void)hipFree(c->dscal);
  if (c->mms_S) (void)hipFree(c->mms_S);
  if (c->mms_H) (void)hipFree(c->mms_H);
  if (c->mms_L) (void)hipFree(c->mms_L);
  if (c->mms_C) (void)hipFree(c->mms_C);

  if (c->vred) (void)hipFree(c->vred);
  if (c->hscal) (void)hipHostFree(c->hscal);
  for (int p = 0; p < NDTM_PROF_NCLASS; ++p)
    for (auto& e : c->ev_used[p]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  for (auto& e : c->ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete c;
}

const char* ndtm_last_error(const ndtm_ctx* c) { return c ? c->err.c_str() : "null context"; }

long long ndtm_half_volume(const ndtm_ctx* c) { return c ? c->V / 2 : 0; }

int ndtm_set_gauge(ndtm_ctx* c, const void* U_dev, void* stream) {
  if (!c || !U_dev) return fail(c, NDTM_EINVAL, "set_gauge: null argument");
  NDTM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)36 * c->g.stride;
  const size_t esz[3] = {16, 8, 4};
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 2; ++q) {
      if (!c->U[p][q]) {
        c->U[p][q] = dev_alloc(c, n * esz[p]);
        if (!c->U[p][q]) return fail(c, NDTM_ENOMEM, "set_gauge: link storage");
        NDTM_HIP(c, hipMemsetAsync(c->U[p][q], 0, n * esz[p], st));
      }
    }
  launch_pack_gauge(c->g, static_cast<const double2*>(U_dev), (double2*)c->U[0][0], (double2*)c->U[0][1],
                    (float2*)c->U[1][0], (float2*)c->U[1][1], (__half2*)c->U[2][0], (__half2*)c->U[2][1],
                    st);
  NDTM_HIP(c, hipGetLastError());
  // SU(3) check: the stencil rebuilds the third row of each link when every
  // stored third row equals conj(row 0 x row 1) to 1e-14
  {
    const int nb = launch_su3_check(c->V, static_cast<const double2*>(U_dev), c->partials, st);
    std::vector<double> part(nb);
    NDTM_HIP(c, hipMemcpyAsync(part.data(), c->partials, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    NDTM_HIP(c, hipStreamSynchronize(st));
    double dev = 0;
    for (double v : part) dev = std::isfinite(v) ? std::max(dev, v) : 1e300;
    c->op.recon12 = dev <= 1e-14 ? 1 : 0;
    c->su3_dev = dev;
  }
  // SU(3) fields: the FP64 stencil reads eight parameters per link, unless some link's
  // first row is too close to (u, 0, 0) for the rebuild's division (unit links, for one)
  c->op.u8[0] = c->op.u8[1] = nullptr;
  if (c->op.recon12) {
    const size_t n8 = (size_t)16 * c->g.stride * sizeof(double2);
    double mn = 1.0;
    for (int q = 0; q < 2; ++q) {
      if (!c->U8[q]) c->U8[q] = dev_alloc(c, n8);
      if (!c->U8[q]) return fail(c, NDTM_ENOMEM, "set_gauge: link storage");
      const int nb = launch_pack_r8(c->g, (const double2*)c->U[P64][q], (double2*)c->U8[q], c->partials, st);
      std::vector<double> part(nb);
      NDTM_HIP(c, hipMemcpyAsync(part.data(), c->partials, nb * sizeof(double), hipMemcpyDeviceToHost, st));
      NDTM_HIP(c, hipStreamSynchronize(st));
      for (double v : part) mn = std::isfinite(v) ? std::min(mn, v) : 0.0;
    }
    if (mn >= kR8MinNorm)
      for (int q = 0; q < 2; ++q) c->op.u8[q] = static_cast<const double2*>(c->U8[q]);
  }
  c->have_gauge = true;
  ndtm_mg_free(c);
  return clover_build(c, st);
}

int ndtm_set_params(ndtm_ctx* c, double kappa, double mubar, double epsbar) {
  if (!c) return NDTM_EINVAL;
  if (!(kappa > 0) || !std::isfinite(mubar) || !std::isfinite(epsbar))
    return fail(c, NDTM_EINVAL, "set_params: kappa must be > 0 and mubar, epsbar finite");
  const double a = 1.0 / (2.0 * kappa);
  const double den = a * a + mubar * mubar - epsbar * epsbar;
  if (den == 0.0) return fail(c, NDTM_EINVAL, "set_params: a^2 + mubar^2 - epsbar^2 == 0");
  c->kappa = kappa;
  c->mubar = mubar;
  c->epsbar = epsbar;
  c->op.a = a;
  c->op.mubar = mubar;
  c->op.epsbar = epsbar;
  c->op.inv_den = 1.0 / den;
  c->have_params = true;
  ndtm_mg_free(c);
  return clover_build(c, nullptr);
}

int ndtm_set_shifts(ndtm_ctx* c, int n, const double* sigma) {
  if (!c) return NDTM_EINVAL;
  if (n < 1 || n > NDTM_MAX_SHIFTS || !sigma) return fail(c, NDTM_EINVAL, "set_shifts: 1..16 shifts");
  for (int i = 0; i < n; ++i) {
    if (!(sigma[i] > 0) || !std::isfinite(sigma[i])) return fail(c, NDTM_EINVAL, "set_shifts: sigma > 0");
    for (int j = 0; j < i; ++j)
      if (sigma[j] == sigma[i]) return fail(c, NDTM_EINVAL, "set_shifts: shifts must be distinct");
  }
  c->shifts.assign(sigma, sigma + n);
  return NDTM_OK;
}

int ndtm_apply(ndtm_ctx* c, int op, int prec, void* y_dev, const void* x_dev, double param, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!y_dev || !x_dev || y_dev == x_dev) return fail(c, NDTM_EINVAL, "apply: null or aliased pointers");
  if (prec < 0 || prec > 3) return fail(c, NDTM_EINVAL, "apply: bad precision");
  if (!c->have_gauge || !c->have_params) return fail(c, NDTM_ESTATE, "apply: set_gauge and set_params first");
  NDTM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double2* x = static_cast<const double2*>(x_dev);
  double2* y = static_cast<double2*>(y_dev);
  // NDTM_PREC_F32_H16 (= P32H): FP32 fields, the stencil on the FP16 links
  const int fp = prec == P32H ? P32 : prec;
  HalfField X = half_field(c, "ap_x", fp), Y = half_field(c, "ap_y", fp), T = half_field(c, "ap_t", fp);
  if (!X.v || !Y.v || !T.v) return fail(c, NDTM_ENOMEM, "apply: workspace");
  switch (op) {
    case NDTM_OP_QHAT:
      launch_pack_half(c->g, x, X, st);
      apply_qhat(c, prec, Y, X, T, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_QHAT2: {
      HalfField U = half_field(c, "ap_u", fp);
      if (!U.v) return fail(c, NDTM_ENOMEM, "apply: workspace");
      launch_pack_half(c->g, x, X, st);
      apply_qhat2(c, prec, Y, X, U, T, param, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    }
    case NDTM_OP_SHAT_SHIFT:
      launch_pack_half(c->g, x, X, st);
      apply_sshift(c, prec, Y, X, T, param, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_DFULL: {
      HalfField Ye = half_field(c, "ap_ye", fp);
      if (!Ye.v) return fail(c, NDTM_ENOMEM, "apply: workspace");
      launch_pack_full(c->g, x, T, X, st);
      apply_dfull(c, prec, Ye, Y, T, X, param, st);
      launch_unpack_full(c->g, Ye, Y, y, st);
      break;
    }
    case NDTM_OP_HOP_EO:
      launch_pack_half(c->g, x, X, st);
      hop(c, prec, EPI_PLAIN, RED_NONE, 0, X, Y, nullptr, nullptr, 0, 0, 0, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    case NDTM_OP_HOP_OE:
      launch_pack_half(c->g, x, X, st);
      hop(c, prec, EPI_PLAIN, RED_NONE, 1, X, Y, nullptr, nullptr, 0, 0, 0, nullptr, st);
      launch_unpack_half(c->g, Y, y, st);
      break;
    default:
      return fail(c, NDTM_EINVAL, "apply: unknown operator");
  }
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_set_stencil_tile(ndtm_ctx* c, int bz, int by) {
  if (!c) return NDTM_EINVAL;
  if (bz < 0 || (bz > 0 && c->g.Lz % bz != 0) || by < 0 || (by > 0 && c->g.Ly % by != 0))
    return fail(c, NDTM_EINVAL, "set_stencil_tile: bz, by must be 0 or divide Lz, Ly");
  c->op.chunk = bz;
  c->op.chunk_y = by;
  return NDTM_OK;
}

int ndtm_stream_bandwidth(ndtm_ctx* c, size_t bytes, int reps, double* copy_gbs, double* read_gbs,
                          double* write_gbs) {
  if (!c) return NDTM_EINVAL;
  if (bytes < (1u << 20) || (bytes & 15) || reps < 1 || !copy_gbs || !read_gbs || !write_gbs)
    return fail(c, NDTM_EINVAL, "stream_bandwidth: bytes >= 1 MiB, multiple of 16; reps >= 1");
  NDTM_HIP(c, hipSetDevice(c->device));
  void *a = nullptr, *b = nullptr;
  unsigned* sink = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess || hipMalloc(&sink, 64) != hipSuccess) {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    return fail(c, NDTM_ENOMEM, "stream_bandwidth: buffers");
  }
  (void)hipMemset(a, 0x5a, bytes);
  (void)hipMemset(b, 0, bytes);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double* out[3] = {copy_gbs, read_gbs, write_gbs};
  for (int kind = 0; kind < 3; ++kind) {
    for (int w = 0; w < 2; ++w) launch_stream(kind, a, b, bytes, sink, nullptr);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r) launch_stream(kind, a, b, bytes, sink, nullptr);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double moved = (kind == 0 ? 2.0 : 1.0) * (double)bytes * reps;
    *out[kind] = ms > 0 ? moved / (ms * 1e-3) / 1e9 : 0.0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(sink);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_profile_enable(ndtm_ctx* c, int on) {
  if (!c) return NDTM_EINVAL;
  c->prof_mask = on;
  if (on) {
    // a pool of event pairs made now, outside the region the caller times
    NDTM_HIP(c, hipSetDevice(c->device));
    while (c->ev_free.size() < 2048) {
      std::pair<hipEvent_t, hipEvent_t> e;
      NDTM_HIP(c, hipEventCreate(&e.first));
      NDTM_HIP(c, hipEventCreate(&e.second));
      c->ev_free.push_back(e);
    }
  }
  return NDTM_OK;
}

int ndtm_profile_read(ndtm_ctx* c, int cls, double* total_ms, long long* launches, double* alg_bytes,
                      int reset) {
  if (!c || cls < 0 || cls >= NDTM_PROF_NCLASS) return NDTM_EINVAL;
  NDTM_HIP(c, hipSetDevice(c->device));
  for (auto& e : c->ev_used[cls]) {
    NDTM_HIP(c, hipEventSynchronize(e.second));
    float ms = 0;
    NDTM_HIP(c, hipEventElapsedTime(&ms, e.first, e.second));
    c->prof_ms[cls] += ms;
    c->prof_n[cls] += 1;
    c->ev_free.push_back(e);
  }
  c->ev_used[cls].clear();
  if (total_ms) *total_ms = c->prof_ms[cls];
  if (launches) *launches = c->prof_n[cls];
  if (alg_bytes) *alg_bytes = c->prof_bytes[cls];
  if (reset) {
    c->prof_ms[cls] = 0;
    c->prof_n[cls] = 0;
    c->prof_bytes[cls] = 0;
    c->prof_moved[cls] = 0;
  }
  return NDTM_OK;
}

int ndtm_profile_moved(const ndtm_ctx* c, int cls, double* moved_bytes) {
  if (!c || cls < 0 || cls >= NDTM_PROF_NCLASS || !moved_bytes) return NDTM_EINVAL;
  *moved_bytes = c->prof_moved[cls];
  return NDTM_OK;
}

}  // extern "C"
