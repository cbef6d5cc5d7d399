// Learned initial-guess proposer: weights, training, inference and the sample
// preparation from solved vectors; the solve-time choice between the network's
// proposal and the Lagrange guess.
//
// A proposal is c = l + tau y over the converged solutions (l the Lagrange
// coefficients, tau = ||r_L|| / ||b||, y the network output), so it stays a mix
// of converged solutions.  Its relative loss 1 + 2 h.y + y.G.y is exact given
// the Gram matrix of [b, x_1..x_K], the Lagrange residual r_L and r_L's
// overlaps with b and the x_i (appendix B: the residual of a combination of
// solutions is the same combination of w_i = -b + (sigma_i - sigma_t) x_i
// added to b).  The network's proposal is used only when this predicted
// residual is below the Lagrange residual; otherwise Lagrange is the fallback.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ctx.h"
#include "mlp.h"
#include "vec.h"

namespace ndtm {

struct MLPData {
  float* W = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  void* Wb = nullptr;     // BF16 copy for inference
  float* gout = nullptr;
  float* hist = nullptr;  // mean loss per training step
  int hist_cap = 0;
  int t = 0;              // Adam step counter
  bool loaded = false;
  // batch buffers
  float *feat = nullptr, *mask = nullptr, *G = nullptr, *h = nullptr, *y = nullptr, *loss = nullptr,
        *gbuf = nullptr;
  int cap = 0;
};

static void mlp_release_batch(ndtm_ctx* c, MLPData* D) {
  for (float** p : {&D->feat, &D->mask, &D->G, &D->h, &D->y, &D->loss, &D->gbuf})
    if (*p) {
      dev_free(c, *p);
      *p = nullptr;
    }
  D->cap = 0;
}

template <class T>
static bool mlp_get(ndtm_ctx* c, T** p, size_t bytes) {
  *p = static_cast<T*>(dev_alloc(c, bytes));
  return *p != nullptr;
}

static int mlp_ensure(ndtm_ctx* c) {
  if (c->mlp) return NDTM_OK;
  MLPData* D = new MLPData();
  c->mlp = D;
  const size_t n = kMlpNParam * sizeof(float);
  if (!mlp_get(c, &D->W, n) || !mlp_get(c, &D->m, n) || !mlp_get(c, &D->v, n) || !mlp_get(c, &D->gout, n) ||
      !mlp_get(c, &D->Wb, kMlpNParam * 2))
    return fail(c, NDTM_ENOMEM, "mlp: weights");
  (void)hipMemset(D->m, 0, n);
  (void)hipMemset(D->v, 0, n);
  return NDTM_OK;
}

static int mlp_batch(ndtm_ctx* c, int B) {
  MLPData* D = c->mlp;
  if (D->cap >= B) return NDTM_OK;
  mlp_release_batch(c, D);
  const size_t b = (size_t)B;
  if (!mlp_get(c, &D->feat, b * kMlpNFeat * 4) || !mlp_get(c, &D->mask, b * kMlpKMax * 4) ||
      !mlp_get(c, &D->G, b * kMlpKMax * kMlpKMax * 4) || !mlp_get(c, &D->h, b * kMlpKMax * 4) ||
      !mlp_get(c, &D->y, b * kMlpKMax * 4) || !mlp_get(c, &D->loss, b * 4) || !mlp_get(c, &D->gbuf, b * kMlpNParam * 4))
    return fail(c, NDTM_ENOMEM, "mlp: batch buffers");
  D->cap = B;
  return NDTM_OK;
}

static int mlp_upload(ndtm_ctx* c, int B, const float* feat, const float* mask, const float* G, const float* h,
                      hipStream_t st) {
  MLPData* D = c->mlp;
  const size_t b = (size_t)B;
  NDTM_HIP(c, hipMemcpyAsync(D->feat, feat, b * kMlpNFeat * 4, hipMemcpyHostToDevice, st));
  if (mask) NDTM_HIP(c, hipMemcpyAsync(D->mask, mask, b * kMlpKMax * 4, hipMemcpyHostToDevice, st));
  else NDTM_HIP(c, hipMemsetAsync(D->mask, 0, b * kMlpKMax * 4, st));
  if (G) NDTM_HIP(c, hipMemcpyAsync(D->G, G, b * kMlpKMax * kMlpKMax * 4, hipMemcpyHostToDevice, st));
  else NDTM_HIP(c, hipMemsetAsync(D->G, 0, b * kMlpKMax * kMlpKMax * 4, st));
  if (h) NDTM_HIP(c, hipMemcpyAsync(D->h, h, b * kMlpKMax * 4, hipMemcpyHostToDevice, st));
  else NDTM_HIP(c, hipMemsetAsync(D->h, 0, b * kMlpKMax * 4, st));
  return NDTM_OK;
}

static std::vector<double> lagrange_coef(const std::vector<double>& nodes, double t) {
  const size_t k = nodes.size();
  std::vector<double> l(k, 1.0);
  for (size_t i = 0; i < k; ++i)
    for (size_t j = 0; j < k; ++j)
      if (j != i) l[i] *= (t - nodes[j]) / (nodes[i] - nodes[j]);
  return l;
}

struct MlpSample {
  float feat[kMlpNFeat];
  float mask[kMlpKMax];
  float G[kMlpKMax * kMlpKMax];
  float h[kMlpKMax];
  double Gd[kMlpKMax * kMlpKMax];  // FP64 copies for the predicted residual
  double hd[kMlpKMax];
  int slot[kMlpKMax];
  std::vector<double> lag;
  double tau = 0, rL2 = 0, bb = 0;
};

// Builds one sample from FP64 internal fields: x_L and r_L = b - (Q^2 + sig_t) x_L,
// Gram of [b, x_1..x_K] and the overlaps with r_L, then features and (G, h).
static int mlp_prepare(ndtm_ctx* c, const std::vector<double>& nodes, const std::vector<HalfField>& xs,
                       double sig_t, const HalfField& b, MlpSample* S, hipStream_t st) {
  const int K = (int)nodes.size();
  if (K < 1 || K > kMlpKMax) return fail(c, NDTM_EINVAL, "mlp sample: 1..11 converged solutions");
  const size_t n = half_elems(c);
  S->lag = lagrange_coef(nodes, sig_t);
  HalfField xl = half_field(c, "ml_xl", P64), rl = half_field(c, "ml_rl", P64);
  if (!xl.v || !rl.v) return fail(c, NDTM_ENOMEM, "mlp sample: workspace");
  std::vector<const double2*> V(K);
  std::vector<double2> cc(K);
  for (int i = 0; i < K; ++i) {
    V[i] = (const double2*)xs[i].v;
    cc[i] = make_double2(S->lag[i], 0.0);
  }
  blas_lincomb((double2*)xl.v, V.data(), cc.data(), K, n, st);
  const double rel = true_residual(c, xl, b, sig_t, rl, st);
  std::vector<const void*> B(K + 1);
  B[0] = b.v;
  for (int i = 0; i < K; ++i) B[1 + i] = xs[i].v;
  double* d = c->dscal + 1024;  // (K+1) Gram columns (i <= j) + the r_L overlaps, complex
  for (int j = 0; j <= K; ++j) vmultidot(P64, B.data(), j + 1, B[j], n, c->vred, d + 2 * (K + 1) * j, st);
  vmultidot(P64, B.data(), K + 1, rl.v, n, c->vred, d + 2 * (K + 1) * (K + 1), st);
  NDTM_HIP(c, hipMemcpyAsync(c->hscal, d, 2 * (K + 1) * (K + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
  NDTM_HIP(c, hipStreamSynchronize(st));
  const double* h = c->hscal;
  // M[i][j] = <B_i, B_j>: column j holds <B_i, B_j> for i <= j; the real part is symmetric
  auto Mre = [&](int i, int j) { return i <= j ? h[2 * ((K + 1) * j + i)] : h[2 * ((K + 1) * i + j)]; };
  auto hre = [&](int i) { return h[2 * ((K + 1) * (K + 1) + i)]; };
  S->bb = Mre(0, 0);
  S->rL2 = rel * rel * S->bb;
  S->tau = rel;
  double gamma = 0;
  for (double l : S->lag) gamma += std::fabs(l);
  std::memset(S->feat, 0, sizeof(S->feat));
  std::memset(S->mask, 0, sizeof(S->mask));
  std::memset(S->G, 0, sizeof(S->G));
  std::memset(S->h, 0, sizeof(S->h));
  std::memset(S->Gd, 0, sizeof(S->Gd));
  std::memset(S->hd, 0, sizeof(S->hd));
  const int near = K - 1;
  std::vector<double> nx(K), dl(K);
  for (int i = 0; i < K; ++i) {
    nx[i] = std::sqrt(std::max(Mre(1 + i, 1 + i), 0.0));
    dl[i] = nodes[i] - sig_t;
  }
  for (int i = 0; i < K; ++i) {
    const int j = near - i;
    S->slot[i] = j;
    const double cosv = Mre(1 + i, 1 + near) / (nx[i] * nx[near]);
    float* f = S->feat + j * 5;
    f[0] = (float)(std::log10(nodes[i] / sig_t) / 5.0);
    f[1] = (float)(S->lag[i] / gamma);
    f[2] = (float)(nx[i] / nx[near]);
    f[3] = (float)(std::log10(std::max(1.0 - cosv, 1e-12)) / 12.0);
    f[4] = 1.0f;
    S->mask[j] = 1.0f;
  }
  float* g = S->feat + kMlpKMax * 5;
  g[0] = (float)(std::log10(sig_t) / 5.0);
  g[1] = (float)K / (float)kMlpKMax;
  g[2] = (float)std::log10(gamma);
  g[3] = (float)(std::log10(std::max(S->tau, 1e-300)) / 10.0);
  const double sh = std::sqrt(S->rL2 * S->bb);
  for (int i = 0; i < K; ++i) {
    const double hw = -hre(0) + dl[i] * hre(1 + i);
    S->hd[S->slot[i]] = sh > 0 ? hw / sh : 0.0;
    for (int k = 0; k < K; ++k) {
      const double gw = Mre(0, 0) - dl[k] * Mre(0, 1 + k) - dl[i] * Mre(1 + i, 0) + dl[i] * dl[k] * Mre(1 + i, 1 + k);
      S->Gd[S->slot[i] * kMlpKMax + S->slot[k]] = gw / S->bb;
    }
  }
  for (int q = 0; q < kMlpKMax * kMlpKMax; ++q) S->G[q] = (float)S->Gd[q];
  for (int q = 0; q < kMlpKMax; ++q) S->h[q] = (float)S->hd[q];
  return NDTM_OK;
}

// Solve-time proposal.  Returns the coefficients over the nodes (node order), the
// predicted relative residual of the network's proposal and of the Lagrange guess.
int guess_mlp(ndtm_ctx* c, const std::vector<double>& nodes, const std::vector<HalfField>& xs, int K, double sig_t,
              const HalfField& b, const std::vector<double>& lag, std::vector<double>* coef, double* pred_mlp,
              double* pred_lag, hipStream_t st) {
  (void)lag;
  MLPData* D = c->mlp;
  if (!D || !D->loaded) return fail(c, NDTM_ESTATE, "guess network: no weights loaded");
  if (K > kMlpKMax) return fail(c, NDTM_EINVAL, "guess network: too many nodes");
  MlpSample S;
  int rc = mlp_prepare(c, nodes, xs, sig_t, b, &S, st);
  if (rc != NDTM_OK) return rc;
  *pred_lag = S.tau;
  if ((rc = mlp_batch(c, 1)) != NDTM_OK) return rc;
  NDTM_HIP(c, hipMemcpyAsync(D->feat, S.feat, sizeof(S.feat), hipMemcpyHostToDevice, st));
  mlp_infer_bf16(D->Wb, D->feat, 1, D->y, st);
  float y[kMlpKMax];
  NDTM_HIP(c, hipMemcpyAsync(y, D->y, sizeof(y), hipMemcpyDeviceToHost, st));
  NDTM_HIP(c, hipStreamSynchronize(st));
  double ym[kMlpKMax];
  for (int j = 0; j < kMlpKMax; ++j) ym[j] = S.mask[j] * (double)y[j];
  double L = 1.0;
  for (int j = 0; j < kMlpKMax; ++j) {
    double gy = 0;
    for (int k = 0; k < kMlpKMax; ++k) gy += S.Gd[j * kMlpKMax + k] * ym[k];
    L += (2.0 * S.hd[j] + gy) * ym[j];
  }
  if (!std::isfinite(L)) return fail(c, NDTM_EBREAKDOWN, "guess network: non-finite output");
  *pred_mlp = L > 0 ? S.tau * std::sqrt(L) : 0.0;
  coef->assign(K, 0.0);
  for (int i = 0; i < K; ++i) (*coef)[i] = S.lag[i] + S.tau * ym[S.slot[i]];
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

void ndtm_mlp_free(ndtm_ctx* c) {
  if (!c || !c->mlp) return;
  MLPData* D = c->mlp;
  mlp_release_batch(c, D);
  for (void* p : {(void*)D->W, (void*)D->m, (void*)D->v, D->Wb, (void*)D->gout, (void*)D->hist}) dev_free(c, p);
  delete D;
  c->mlp = nullptr;
}

int ndtm_mlp_set_weights(ndtm_ctx* c, const float* w, size_t n) {
  if (!c) return NDTM_EINVAL;
  if (!w || n != (size_t)kMlpNParam) return fail(c, NDTM_EINVAL, "mlp_set_weights: need NDTM_MLP_NPARAM floats");
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(w[i])) return fail(c, NDTM_EINVAL, "mlp_set_weights: non-finite weight");
  NDTM_HIP(c, hipSetDevice(c->device));
  int rc = mlp_ensure(c);
  if (rc != NDTM_OK) return rc;
  MLPData* D = c->mlp;
  NDTM_HIP(c, hipMemcpy(D->W, w, n * 4, hipMemcpyHostToDevice));
  NDTM_HIP(c, hipMemset(D->m, 0, n * 4));
  NDTM_HIP(c, hipMemset(D->v, 0, n * 4));
  D->t = 0;
  mlp_make_bf16(D->W, D->Wb, nullptr);
  NDTM_HIP(c, hipDeviceSynchronize());
  D->loaded = true;
  return NDTM_OK;
}

int ndtm_mlp_get_weights(ndtm_ctx* c, float* w, size_t n) {
  if (!c) return NDTM_EINVAL;
  if (!c->mlp || !c->mlp->loaded) return fail(c, NDTM_ESTATE, "mlp_get_weights: no weights");
  if (!w || n != (size_t)kMlpNParam) return fail(c, NDTM_EINVAL, "mlp_get_weights: need NDTM_MLP_NPARAM floats");
  NDTM_HIP(c, hipMemcpy(w, c->mlp->W, n * 4, hipMemcpyDeviceToHost));
  return NDTM_OK;
}

int ndtm_mlp_forward(ndtm_ctx* c, int B, const float* feat, const float* mask, const float* G, const float* h,
                     int bf16, float* y_out, float* loss_out) {
  if (!c) return NDTM_EINVAL;
  if (!c->mlp || !c->mlp->loaded) return fail(c, NDTM_ESTATE, "mlp_forward: no weights");
  if (B < 1 || !feat || !y_out) return fail(c, NDTM_EINVAL, "mlp_forward: bad arguments");
  NDTM_HIP(c, hipSetDevice(c->device));
  int rc = mlp_batch(c, B);
  if (rc != NDTM_OK) return rc;
  if ((rc = mlp_upload(c, B, feat, mask, G, h, nullptr)) != NDTM_OK) return rc;
  MLPData* D = c->mlp;
  if (bf16)
    mlp_infer_bf16(D->Wb, D->feat, B, D->y, nullptr);
  else
    mlp_forward_fp32(D->W, D->feat, D->mask, D->G, D->h, B, D->y, D->loss, nullptr);
  NDTM_HIP(c, hipMemcpy(y_out, D->y, (size_t)B * kMlpKMax * 4, hipMemcpyDeviceToHost));
  if (loss_out && !bf16) NDTM_HIP(c, hipMemcpy(loss_out, D->loss, (size_t)B * 4, hipMemcpyDeviceToHost));
  return NDTM_OK;
}

int ndtm_mlp_grad(ndtm_ctx* c, int B, const float* feat, const float* mask, const float* G, const float* h,
                  float* grad_out, float* mean_loss) {
  if (!c) return NDTM_EINVAL;
  if (!c->mlp || !c->mlp->loaded) return fail(c, NDTM_ESTATE, "mlp_grad: no weights");
  if (B < 1 || !feat || !mask || !G || !h || !grad_out) return fail(c, NDTM_EINVAL, "mlp_grad: bad arguments");
  NDTM_HIP(c, hipSetDevice(c->device));
  int rc = mlp_batch(c, B);
  if (rc != NDTM_OK) return rc;
  if ((rc = mlp_upload(c, B, feat, mask, G, h, nullptr)) != NDTM_OK) return rc;
  MLPData* D = c->mlp;
  mlp_grad_step(D->W, D->m, D->v, D->feat, D->mask, D->G, D->h, B, D->loss, D->gbuf, D->gout, 0, 0.f, 0,
                (float*)c->dscal, nullptr);
  NDTM_HIP(c, hipMemcpy(grad_out, D->gout, kMlpNParam * 4, hipMemcpyDeviceToHost));
  if (mean_loss) NDTM_HIP(c, hipMemcpy(mean_loss, c->dscal, 4, hipMemcpyDeviceToHost));
  return NDTM_OK;
}

int ndtm_mlp_train(ndtm_ctx* c, int B, const float* feat, const float* mask, const float* G, const float* h, int steps,
                   float lr, float* loss_hist) {
  if (!c) return NDTM_EINVAL;
  if (!c->mlp || !c->mlp->loaded) return fail(c, NDTM_ESTATE, "mlp_train: load initial weights first");
  if (B < 1 || steps < 1 || !(lr > 0) || !feat || !mask || !G || !h)
    return fail(c, NDTM_EINVAL, "mlp_train: bad arguments");
  NDTM_HIP(c, hipSetDevice(c->device));
  int rc = mlp_batch(c, B);
  if (rc != NDTM_OK) return rc;
  if ((rc = mlp_upload(c, B, feat, mask, G, h, nullptr)) != NDTM_OK) return rc;
  MLPData* D = c->mlp;
  if (D->hist_cap < steps) {
    dev_free(c, D->hist);
    if (!mlp_get(c, &D->hist, (size_t)steps * 4)) {
      D->hist_cap = 0;
      return fail(c, NDTM_ENOMEM, "mlp_train: history");
    }
    D->hist_cap = steps;
  }
  for (int k = 0; k < steps; ++k) {
    ++D->t;
    mlp_grad_step(D->W, D->m, D->v, D->feat, D->mask, D->G, D->h, B, D->loss, D->gbuf, nullptr, 1, lr, D->t,
                  D->hist + k, nullptr);
  }
  mlp_make_bf16(D->W, D->Wb, nullptr);
  NDTM_HIP(c, hipGetLastError());
  if (loss_hist) NDTM_HIP(c, hipMemcpy(loss_hist, D->hist, (size_t)steps * 4, hipMemcpyDeviceToHost));
  NDTM_HIP(c, hipDeviceSynchronize());
  return NDTM_OK;
}

int ndtm_mlp_sample(ndtm_ctx* c, int K, void* const* x_dev, const double* nodes, double sig_t, const void* b_dev,
                    float* feat, float* mask, float* G, float* h, double* info, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->have_gauge || !c->have_params) return fail(c, NDTM_ESTATE, "mlp_sample: set_gauge and set_params first");
  if (K < 1 || K > kMlpKMax || !x_dev || !nodes || !b_dev || !feat || !mask || !G || !h)
    return fail(c, NDTM_EINVAL, "mlp_sample: bad arguments");
  for (int i = 0; i < K; ++i) {
    if (!x_dev[i] || !(nodes[i] > sig_t) || (i > 0 && !(nodes[i] < nodes[i - 1])))
      return fail(c, NDTM_EINVAL, "mlp_sample: nodes must be descending and above the target");
  }
  NDTM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<HalfField> xs(K);
  for (int i = 0; i < K; ++i) {
    xs[i] = half_field(c, "ms_x" + std::to_string(i), P64);
    if (!xs[i].v) return fail(c, NDTM_ENOMEM, "mlp_sample: workspace");
    launch_pack_half(c->g, static_cast<const double2*>(x_dev[i]), xs[i], st);
  }
  HalfField bf = half_field(c, "ms_b", P64);
  if (!bf.v) return fail(c, NDTM_ENOMEM, "mlp_sample: workspace");
  launch_pack_half(c->g, static_cast<const double2*>(b_dev), bf, st);
  MlpSample S;
  const int first = guess_first_node(std::vector<double>(nodes, nodes + K), sig_t);
  std::vector<double> nd(nodes + first, nodes + K);
  std::vector<HalfField> xk(xs.begin() + first, xs.end());
  int rc = mlp_prepare(c, nd, xk, sig_t, bf, &S, st);
  if (rc != NDTM_OK) return rc;
  std::memcpy(feat, S.feat, sizeof(S.feat));
  std::memcpy(mask, S.mask, sizeof(S.mask));
  std::memcpy(G, S.G, sizeof(S.G));
  std::memcpy(h, S.h, sizeof(S.h));
  if (info) {
    info[0] = S.tau;
    info[1] = S.rL2;
    info[2] = S.bb;
    info[3] = first;
  }
  return NDTM_OK;
}

}  // extern "C"
