// Learned launch-configuration tuner: a small MLP cost model, trained on the GPU
// by the kernels in kernels/mlp.hip on timings the autotuner produced, that
// predicts log(time) for every configuration of an expression signature on a
// shape; the prediction's argmin is the chosen configuration.
//
// Feature vector (23 values): n_ops, n_operands, one-hot dtype (u32 s32 f32 f64),
// log2(1 + rows), log2(1 + cols), n_trans, one-hot reduction (none all dim0 dim1),
// log2 vec, log2 ept, log2 waves, log2 grid_mult, then four launch quantities the
// configuration implies (for contiguous operands on 256 CUs): log2(1 + elements),
// the tiled-family flag, log2(workgroups launched), log2(1 + elements per thread),
// and the tile of the tiled family, log2(tile_r) and log2(tile_c) (0 for flat kernels).
// Inputs and the target are z-scored with the training set's statistics, stored
// with the weights.  A model is an ensemble of networks trained from different
// initial parameters and batch orders; its prediction is their mean.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <random>

#include "core.h"

extern "C" {
hipError_t coot_mlp_k_dense_fwd(const float* X, int B, int K, const float* W, const float* bias, int O, float* Z,
                                float* A, int relu, hipStream_t s);
hipError_t coot_mlp_k_mse_grad(const float* out, const float* y, const float* mask, int B, float inv_count, float* dZ,
                               float* L, float* loss, hipStream_t s);
hipError_t coot_mlp_k_dense_bwd(const float* dZ, const float* A, const float* W, int B, int K, int O, float* dW,
                                float* db, const float* Zp, float* dZp, hipStream_t s);
hipError_t coot_mlp_k_adam(float* P, const float* G, float* M, float* V, int n, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t s);
hipError_t coot_mlp_k_gather(const float* X, const float* y, const float* mask, const int* idx, int B, int K,
                             float* Xb, float* yb, float* mb, hipStream_t s);
}

using namespace coot;

namespace {

void* dmalloc(size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 4)) != hipSuccess) fail(COOT_ENOMEM, "cost-model allocation failed");
  return p;
}

}  // namespace

struct coot_mlp {
  int F = 0, H1 = 0, H2 = 0;
  size_t n = 0;
  float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
  int cap = 0;
  float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Z3 = nullptr, *A3 = nullptr;
  float *dZ3 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *L = nullptr, *loss = nullptr;
  float *Xb = nullptr, *yb = nullptr, *mb = nullptr;
  int* idx = nullptr;
  int idx_cap = 0;
  size_t oW1() const { return 0; }
  size_t ob1() const { return (size_t)H1 * F; }
  size_t oW2() const { return ob1() + H1; }
  size_t ob2() const { return oW2() + (size_t)H2 * H1; }
  size_t oW3() const { return ob2() + H2; }
  size_t ob3() const { return oW3() + H2; }
  void free_acts() {
    for (float* p : {Z1, A1, Z2, A2, Z3, A3, dZ3, dZ2, dZ1, L, Xb, yb, mb})
      if (p) (void)hipFree(p);
    Z1 = A1 = Z2 = A2 = Z3 = A3 = dZ3 = dZ2 = dZ1 = L = Xb = yb = mb = nullptr;
  }
  void ensure(int B) {
    if (B <= cap) return;
    free_acts();
    Z1 = (float*)dmalloc((size_t)B * H1 * 4);
    A1 = (float*)dmalloc((size_t)B * H1 * 4);
    Z2 = (float*)dmalloc((size_t)B * H2 * 4);
    A2 = (float*)dmalloc((size_t)B * H2 * 4);
    Z3 = (float*)dmalloc((size_t)B * 4);
    A3 = (float*)dmalloc((size_t)B * 4);
    dZ3 = (float*)dmalloc((size_t)B * 4);
    dZ2 = (float*)dmalloc((size_t)B * H2 * 4);
    dZ1 = (float*)dmalloc((size_t)B * H1 * 4);
    L = (float*)dmalloc((size_t)B * 4);
    Xb = (float*)dmalloc((size_t)B * F * 4);
    yb = (float*)dmalloc((size_t)B * 4);
    mb = (float*)dmalloc((size_t)B * 4);
    cap = B;
  }
  ~coot_mlp() {
    free_acts();
    for (float* p : {P, G, M, V, loss})
      if (p) (void)hipFree(p);
    if (idx) (void)hipFree(idx);
  }
};

namespace {

void forward(coot_mlp* m, const float* X, int B, hipStream_t s) {
  m->ensure(B);
  const float* P = m->P;
  hip_check(coot_mlp_k_dense_fwd(X, B, m->F, P + m->oW1(), P + m->ob1(), m->H1, m->Z1, m->A1, 1, s), "mlp fwd 1");
  hip_check(coot_mlp_k_dense_fwd(m->A1, B, m->H1, P + m->oW2(), P + m->ob2(), m->H2, m->Z2, m->A2, 1, s), "mlp fwd 2");
  hip_check(coot_mlp_k_dense_fwd(m->A2, B, m->H2, P + m->oW3(), P + m->ob3(), 1, m->Z3, m->A3, 0, s), "mlp fwd 3");
}

void backward(coot_mlp* m, const float* X, const float* y, const float* mask, int B, float inv_count, float* loss,
              hipStream_t s) {
  forward(m, X, B, s);
  float* G = m->G;
  hip_check(coot_mlp_k_mse_grad(m->A3, y, mask, B, inv_count, m->dZ3, m->L, loss, s), "mlp mse");
  hip_check(coot_mlp_k_dense_bwd(m->dZ3, m->A2, m->P + m->oW3(), B, m->H2, 1, G + m->oW3(), G + m->ob3(), m->Z2,
                                 m->dZ2, s),
            "mlp bwd 3");
  hip_check(coot_mlp_k_dense_bwd(m->dZ2, m->A1, m->P + m->oW2(), B, m->H1, m->H2, G + m->oW2(), G + m->ob2(), m->Z1,
                                 m->dZ1, s),
            "mlp bwd 2");
  hip_check(coot_mlp_k_dense_bwd(m->dZ1, X, m->P + m->oW1(), B, m->F, m->H1, G + m->oW1(), G + m->ob1(), nullptr,
                                 nullptr, s),
            "mlp bwd 1");
}

void adam_step(coot_mlp* m, float lr, float b1, float b2, float eps, int t, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, t));
  const float c2 = (float)(1.0 - std::pow((double)b2, t));
  hip_check(coot_mlp_k_adam(m->P, m->G, m->M, m->V, (int)m->n, lr, b1, b2, eps, c1, c2, s), "mlp adam");
}

}  // namespace

extern "C" {

coot_status coot_mlp_create(int32_t n_in, int32_t h1, int32_t h2, const float* params_host, coot_mlp** out) {
  return guarded([&] {
    if (!out || !params_host || n_in <= 0 || h1 <= 0 || h2 <= 0) fail(COOT_EINVAL, "bad MLP arguments");
    auto m = std::make_unique<coot_mlp>();
    m->F = n_in;
    m->H1 = h1;
    m->H2 = h2;
    m->n = (size_t)h1 * n_in + h1 + (size_t)h2 * h1 + h2 + h2 + 1;
    m->P = (float*)dmalloc(m->n * 4);
    m->G = (float*)dmalloc(m->n * 4);
    m->M = (float*)dmalloc(m->n * 4);
    m->V = (float*)dmalloc(m->n * 4);
    m->loss = (float*)dmalloc(4);
    hip_check(hipMemcpy(m->P, params_host, m->n * 4, hipMemcpyHostToDevice), "hipMemcpy");
    hip_check(hipMemset(m->G, 0, m->n * 4), "hipMemset");
    hip_check(hipMemset(m->M, 0, m->n * 4), "hipMemset");
    hip_check(hipMemset(m->V, 0, m->n * 4), "hipMemset");
    *out = m.release();
  });
}

uint32_t coot_mlp_num_params(const coot_mlp* m) { return m ? (uint32_t)m->n : 0; }

coot_status coot_mlp_get_params(const coot_mlp* m, float* host) {
  return guarded([&] {
    if (!m || !host) fail(COOT_EINVAL, "NULL argument");
    hip_check(hipMemcpy(host, m->P, m->n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  });
}

coot_status coot_mlp_get_grads(const coot_mlp* m, float* host) {
  return guarded([&] {
    if (!m || !host) fail(COOT_EINVAL, "NULL argument");
    hip_check(hipMemcpy(host, m->G, m->n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  });
}

coot_status coot_mlp_forward(coot_mlp* m, const float* X, int32_t B, float* out, void* stream) {
  return guarded([&] {
    if (!m || (B && (!X || !out)) || B < 0) fail(COOT_EINVAL, "bad MLP forward arguments");
    if (B == 0) return;
    hipStream_t s = (hipStream_t)stream;
    forward(m, X, B, s);
    hip_check(hipMemcpyAsync(out, m->A3, (size_t)B * 4, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
  });
}

coot_status coot_mlp_backward(coot_mlp* m, const float* X, const float* y, const float* mask, int32_t B,
                              float inv_count, float* loss, void* stream) {
  return guarded([&] {
    if (!m || !X || !y || !mask || B <= 0) fail(COOT_EINVAL, "bad MLP backward arguments");
    backward(m, X, y, mask, B, inv_count, loss, (hipStream_t)stream);
  });
}

coot_status coot_mlp_adam_step(coot_mlp* m, float lr, float beta1, float beta2, float eps, int32_t t, void* stream) {
  return guarded([&] {
    if (!m || t < 1) fail(COOT_EINVAL, "bad Adam arguments");
    adam_step(m, lr, beta1, beta2, eps, t, (hipStream_t)stream);
  });
}

coot_status coot_mlp_train(coot_mlp* m, const float* X, const float* y, const float* mask, const float* mask_host,
                           int32_t N, int32_t batch, int32_t epochs, uint32_t seed, float lr, float* losses_host,
                           void* stream) {
  return guarded([&] {
    if (!m || !X || !y || !mask || !mask_host || N <= 0 || batch <= 0 || epochs < 0) fail(COOT_EINVAL, "bad train arguments");
    hipStream_t s = (hipStream_t)stream;
    if (N > m->idx_cap) {
      if (m->idx) (void)hipFree(m->idx);
      m->idx = (int*)dmalloc((size_t)N * 4);
      m->idx_cap = N;
    }
    m->ensure(batch);
    std::mt19937_64 rng(seed);
    std::vector<int> perm(N);
    const int steps_per_epoch = (N + batch - 1) / batch;
    float* dloss = (float*)dmalloc((size_t)steps_per_epoch * 4);
    std::vector<float> lbuf(steps_per_epoch);
    int t = 0;
    try {
      for (int ep = 0; ep < epochs; ++ep) {
        std::iota(perm.begin(), perm.end(), 0);
        std::shuffle(perm.begin(), perm.end(), rng);
        hip_check(hipMemcpyAsync(m->idx, perm.data(), (size_t)N * 4, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
        for (int st = 0; st < steps_per_epoch; ++st) {
          const int b0 = st * batch, B = std::min(batch, N - b0);
          double cnt = 0;
          for (int r = 0; r < B; ++r) cnt += mask_host[perm[b0 + r]];
          const float inv = cnt > 0 ? (float)(1.0 / cnt) : 0.0f;
          hip_check(coot_mlp_k_gather(X, y, mask, m->idx + b0, B, m->F, m->Xb, m->yb, m->mb, s), "mlp gather");
          backward(m, m->Xb, m->yb, m->mb, B, inv, dloss + st, s);
          adam_step(m, lr, 0.9f, 0.999f, 1e-8f, ++t, s);
        }
        hip_check(hipMemcpyAsync(lbuf.data(), dloss, (size_t)steps_per_epoch * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");  // perm is rewritten next epoch
        if (losses_host) {
          double acc = 0;
          for (float v : lbuf) acc += v;
          losses_host[ep] = (float)(acc / steps_per_epoch);
        }
      }
    } catch (...) {
      (void)hipFree(dloss);
      throw;
    }
    (void)hipFree(dloss);
  });
}

void coot_mlp_release(coot_mlp* m) { delete m; }

}  // extern "C"

// ---------------------------------------------------------------------------------
// Cost model
// ---------------------------------------------------------------------------------
static constexpr int kNF = 23;
static constexpr int kFeatCUs = 256;  // CU count the launch-quantity features assume
static constexpr int kMaxModels = 16;

struct coot_costmodel {
  std::vector<coot_mlp*> mlps;
  float mean[kNF], stdv[kNF];
  float y_mean = 0, y_std = 1;
  float* d_feat = nullptr;
  float* d_out = nullptr;
  int cap = 0;
  ~coot_costmodel() {
    for (auto* m : mlps) delete m;
    if (d_feat) (void)hipFree(d_feat);
    if (d_out) (void)hipFree(d_out);
  }
};

namespace {

void features_of(const Expr& e, int64_t R, int64_t C, int red, const coot_launch_cfg& c, float* f) {
  if (dtype_is_half(e.dtype)) fail(COOT_EUNSUPPORTED, "the cost model covers u32, s32, f32 and f64 expressions");
  int n_ops = 0, n_trans = 0;
  std::vector<bool> seen(e.slots.size(), false);
  int n_operands = 0;
  for (auto& o : e.ops) {
    if (o.code == COOT_OP_LOAD) {
      if (!seen[o.arg]) {
        seen[o.arg] = true;
        ++n_operands;
      }
    } else if (o.code != COOT_OP_SCALAR) {
      ++n_ops;
      if (o.code == COOT_OP_TRANS) ++n_trans;
    }
  }
  int k = 0;
  f[k++] = (float)n_ops;
  f[k++] = (float)n_operands;
  for (int d : {COOT_U32, COOT_S32, COOT_F32, COOT_F64}) f[k++] = e.dtype == d ? 1.0f : 0.0f;
  f[k++] = (float)std::log2(1.0 + (double)R);
  f[k++] = (float)std::log2(1.0 + (double)C);
  f[k++] = (float)n_trans;
  for (int r = 0; r < 4; ++r) f[k++] = red == r ? 1.0f : 0.0f;  // 0 none, 1 all, 2 dim0, 3 dim1
  f[k++] = (float)std::log2((double)c.vec);
  f[k++] = (float)std::log2((double)c.ept);
  f[k++] = (float)std::log2((double)c.waves);
  f[k++] = (float)std::log2((double)c.grid_mult);
  // launch quantities: the tiled family (transposed leaves or a dimension sum) runs
  // 256 threads per tile_r x tile_c tile (64 x 64 when the configuration names none);
  // the flat family 64 * waves threads, each taking ept groups of vec elements per pass
  const double n = (double)R * (double)C;
  const bool tiled = e.n_p1 > 0 || red >= 2;
  const double cap = (double)c.grid_mult * kFeatCUs;
  const double tr = c.tile_r ? c.tile_r : 64, tcl = c.tile_c ? c.tile_c : 64;
  double grid, threads;
  if (tiled) {
    grid = std::min(std::ceil((double)R / tr) * std::ceil((double)C / tcl), cap);
    threads = 256;
  } else {
    threads = 64.0 * c.waves;
    grid = std::min(std::ceil(std::max(1.0, std::ceil(n / c.vec)) / (threads * c.ept)), cap);
  }
  grid = std::max(1.0, grid);
  f[k++] = (float)std::log2(1.0 + n);
  f[k++] = tiled ? 1.0f : 0.0f;
  f[k++] = (float)std::log2(grid);
  f[k++] = (float)std::log2(1.0 + n / (grid * threads));
  f[k++] = tiled ? (float)std::log2(tr) : 0.0f;
  f[k++] = tiled ? (float)std::log2(tcl) : 0.0f;
}

}  // namespace

extern "C" {

coot_status coot_costmodel_features(const coot_expr* h, int64_t n_rows, int64_t n_cols, int32_t red,
                                    const coot_launch_cfg* cfgs, uint32_t n, float* out) {
  return guarded([&] {
    if (!h || (n && (!cfgs || !out))) fail(COOT_EINVAL, "NULL argument");
    if (red < 0 || red > 3) fail(COOT_EINVAL, "reduction code must be 0..3");
    for (uint32_t i = 0; i < n; ++i) features_of(*h->e, n_rows, n_cols, red, cfgs[i], out + (size_t)i * kNF);
  });
}

coot_status coot_costmodel_train(const float* feats, const float* target, const float* mask, int32_t N,
                                 const float* init_params, int32_t n_models, int32_t h1, int32_t h2, int32_t epochs,
                                 int32_t batch, uint32_t seed, float lr, float* losses, void* stream,
                                 coot_costmodel** out) {
  return guarded([&] {
    if (!feats || !target || !mask || !init_params || !out || N <= 1) fail(COOT_EINVAL, "bad training arguments");
    if (n_models < 1 || n_models > kMaxModels) fail(COOT_EINVAL, "n_models must be 1..16");
    auto cm = std::make_unique<coot_costmodel>();
    // z-score statistics of the training set (binary64 accumulation)
    for (int j = 0; j < kNF; ++j) {
      double s = 0, s2 = 0;
      for (int i = 0; i < N; ++i) s += feats[(size_t)i * kNF + j];
      const double mu = s / N;
      for (int i = 0; i < N; ++i) {
        const double d = feats[(size_t)i * kNF + j] - mu;
        s2 += d * d;
      }
      const double sd = std::sqrt(s2 / N);
      cm->mean[j] = (float)mu;
      cm->stdv[j] = sd > 1e-12 ? (float)sd : 1.0f;
    }
    double ys = 0, ys2 = 0, cnt = 0;
    for (int i = 0; i < N; ++i)
      if (mask[i] > 0) {
        ys += target[i];
        cnt += 1;
      }
    const double ym = cnt > 0 ? ys / cnt : 0;
    for (int i = 0; i < N; ++i)
      if (mask[i] > 0) ys2 += (target[i] - ym) * (target[i] - ym);
    const double ysd = cnt > 1 ? std::sqrt(ys2 / cnt) : 1.0;
    cm->y_mean = (float)ym;
    cm->y_std = ysd > 1e-12 ? (float)ysd : 1.0f;
    std::vector<float> Xn((size_t)N * kNF), yn(N);
    for (int i = 0; i < N; ++i) {
      for (int j = 0; j < kNF; ++j) Xn[(size_t)i * kNF + j] = (feats[(size_t)i * kNF + j] - cm->mean[j]) / cm->stdv[j];
      yn[i] = mask[i] > 0 ? (float)((target[i] - ym) / cm->y_std) : 0.0f;
    }
    hipStream_t s = (hipStream_t)stream;
    float* dX = (float*)dmalloc(Xn.size() * 4);
    float* dy = (float*)dmalloc((size_t)N * 4);
    float* dm = (float*)dmalloc((size_t)N * 4);
    try {
      hip_check(hipMemcpy(dX, Xn.data(), Xn.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
      hip_check(hipMemcpy(dy, yn.data(), (size_t)N * 4, hipMemcpyHostToDevice), "hipMemcpy");
      hip_check(hipMemcpy(dm, mask, (size_t)N * 4, hipMemcpyHostToDevice), "hipMemcpy");
      const size_t np = (size_t)h1 * kNF + h1 + (size_t)h2 * h1 + h2 + h2 + 1;
      std::vector<float> ls(std::max(1, epochs));
      for (int k = 0; k < n_models; ++k) {
        coot_mlp* m = nullptr;
        coot_status st = coot_mlp_create(kNF, h1, h2, init_params + k * np, &m);
        if (st != COOT_OK) fail(st, last_error());
        cm->mlps.push_back(m);
        // network k: its own initial parameters and batch order (seed + k)
        st = coot_mlp_train(m, dX, dy, dm, mask, N, batch, epochs, seed + (uint32_t)k, lr, ls.data(), s);
        if (st != COOT_OK) fail(st, last_error());
        if (losses)
          for (int e = 0; e < epochs; ++e) losses[e] = (k == 0 ? 0.0f : losses[e]) + ls[e] / (float)n_models;
      }
    } catch (...) {
      (void)hipFree(dX);
      (void)hipFree(dy);
      (void)hipFree(dm);
      throw;
    }
    (void)hipFree(dX);
    (void)hipFree(dy);
    (void)hipFree(dm);
    *out = cm.release();
  });
}

// Predicted time (microseconds) of each configuration, and the argmin (lowest index on ties).
coot_status coot_costmodel_predict(coot_costmodel* cm, const coot_expr* h, int64_t n_rows, int64_t n_cols,
                                   int32_t red, const coot_launch_cfg* cfgs, uint32_t n, float* pred_us,
                                   uint32_t* best, void* stream) {
  return guarded([&] {
    if (!cm || !h || !cfgs || n == 0) fail(COOT_EINVAL, "bad predict arguments");
    std::vector<float> f((size_t)n * kNF);
    for (uint32_t i = 0; i < n; ++i) {
      features_of(*h->e, n_rows, n_cols, red, cfgs[i], &f[(size_t)i * kNF]);
      for (int j = 0; j < kNF; ++j) f[(size_t)i * kNF + j] = (f[(size_t)i * kNF + j] - cm->mean[j]) / cm->stdv[j];
    }
    if ((int)n > cm->cap) {
      if (cm->d_feat) (void)hipFree(cm->d_feat);
      if (cm->d_out) (void)hipFree(cm->d_out);
      cm->d_feat = (float*)dmalloc(f.size() * 4);
      cm->d_out = (float*)dmalloc((size_t)n * 4);
      cm->cap = (int)n;
    }
    hipStream_t s = (hipStream_t)stream;
    hip_check(hipMemcpyAsync(cm->d_feat, f.data(), f.size() * 4, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    std::vector<float> y(n, 0.0f), yk(n);
    for (auto* m : cm->mlps) {
      forward(m, cm->d_feat, (int)n, s);
      hip_check(hipMemcpyAsync(yk.data(), m->A3, (size_t)n * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      for (uint32_t i = 0; i < n; ++i) y[i] += yk[i] / (float)cm->mlps.size();
    }
    uint32_t bi = 0;
    for (uint32_t i = 0; i < n; ++i) {
      const float us = std::exp(y[i] * cm->y_std + cm->y_mean);
      if (pred_us) pred_us[i] = us;
      if (y[i] < y[bi]) bi = i;
    }
    if (best) *best = bi;
  });
}

coot_status coot_costmodel_save(const coot_costmodel* cm, const char* path) {
  return guarded([&] {
    if (!cm || !path) fail(COOT_EINVAL, "NULL argument");
    if (cm->mlps.empty()) fail(COOT_EINVAL, "empty cost model");
    const coot_mlp* m0 = cm->mlps[0];
    std::ofstream f(path, std::ios::binary);
    if (!f) fail(COOT_EINVAL, std::string("cannot write ") + path);
    const char magic[8] = {'C', 'O', 'O', 'T', 'M', 'L', 'P', '2'};
    const int32_t dims[4] = {m0->F, m0->H1, m0->H2, (int32_t)cm->mlps.size()};
    f.write(magic, 8);
    f.write((const char*)dims, sizeof dims);
    f.write((const char*)cm->mean, sizeof cm->mean);
    f.write((const char*)cm->stdv, sizeof cm->stdv);
    f.write((const char*)&cm->y_mean, 4);
    f.write((const char*)&cm->y_std, 4);
    for (const auto* m : cm->mlps) {
      std::vector<float> p(m->n);
      hip_check(hipMemcpy(p.data(), m->P, p.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy");
      f.write((const char*)p.data(), (std::streamsize)(p.size() * 4));
    }
    if (!f) fail(COOT_EINVAL, std::string("write failed: ") + path);
  });
}

coot_status coot_costmodel_load(const char* path, coot_costmodel** out) {
  return guarded([&] {
    if (!path || !out) fail(COOT_EINVAL, "NULL argument");
    std::ifstream f(path, std::ios::binary);
    if (!f) fail(COOT_EINVAL, std::string("cannot read ") + path);
    char magic[8];
    int32_t dims[4];
    f.read(magic, 8);
    f.read((char*)dims, sizeof dims);
    if (!f || std::memcmp(magic, "COOTMLP2", 8) != 0 || dims[0] != kNF || dims[1] <= 0 || dims[2] <= 0 ||
        dims[1] > 4096 || dims[2] > 4096 || dims[3] < 1 || dims[3] > kMaxModels)
      fail(COOT_EINVAL, "not a cost-model file");
    auto cm = std::make_unique<coot_costmodel>();
    f.read((char*)cm->mean, sizeof cm->mean);
    f.read((char*)cm->stdv, sizeof cm->stdv);
    f.read((char*)&cm->y_mean, 4);
    f.read((char*)&cm->y_std, 4);
    const size_t n = (size_t)dims[1] * dims[0] + dims[1] + (size_t)dims[2] * dims[1] + dims[2] + dims[2] + 1;
    for (int k = 0; k < dims[3]; ++k) {
      std::vector<float> p(n);
      f.read((char*)p.data(), (std::streamsize)(n * 4));
      if (!f) fail(COOT_EINVAL, "truncated cost-model file");
      coot_mlp* m = nullptr;
      coot_status st = coot_mlp_create(dims[0], dims[1], dims[2], p.data(), &m);
      if (st != COOT_OK) fail(st, last_error());
      cm->mlps.push_back(m);
    }
    *out = cm.release();
  });
}

void coot_costmodel_release(coot_costmodel* cm) { delete cm; }

// The cost model's pick replaces the library default only when predicted this much faster.
constexpr float kCostModelMargin = 0.05f;

// Choose a configuration: 0 DEFAULT, 1 EXHAUSTIVE (time all), 2 MLP (cost-model argmin, then timed).
coot_status coot_tune(coot_expr* h, const coot_operand* operands, const double* scalars, coot_operand* out,
                      int32_t mode, int32_t dim, int32_t policy, coot_costmodel* cm, coot_launch_cfg* best,
                      float* best_us, void* stream) {
  return guarded([&] {
    if (!h || !out || !best) fail(COOT_EINVAL, "NULL argument");
    int32_t fam = 0;
    coot_status st = coot_tune_prepare(h, operands, mode, dim, &fam);
    if (st != COOT_OK) fail(st, last_error());
    std::vector<coot_launch_cfg> space(coot_tune_space(fam, nullptr, 0));
    coot_tune_space(fam, space.data(), (uint32_t)space.size());
    std::vector<coot_launch_cfg> cand;
    // the configuration the library launches without a tuner, as an entry of the space
    auto library_default = [&]() {
      int64_t R, C;
      infer_shape(*h->e, operands, &R, &C);
      coot_launch_cfg d = default_cfg(fam == 0 ? FAM_FLAT : FAM_TILE, mode, is_dim_kind(mode) ? dim : -1, h->e->dtype,
                                      R * C);
      if (!d.ept) d.ept = 1;  // the tiled family's configurations carry ept 1
      if (fam == 1 && !d.tile_r) {  // the library's tile (default_tile)
        int tr = 0, tc = 0;
        default_tile(*h->e, mode, is_dim_kind(mode) ? dim : -1, R * C, &tr, &tc);
        d.tile_r = (uint16_t)tr;
        d.tile_c = (uint16_t)tc;
        if (d.vec > tile_vec_cap(d.tile_r, d.tile_c)) d.vec = (uint16_t)tile_vec_cap(d.tile_r, d.tile_c);
      }
      return d;
    };
    if (policy == 0) {
      cand.push_back(library_default());
    } else if (policy == 1) {
      cand = space;
      if (dtype_is_half(h->e->dtype))  // 16-byte groups of 16-bit elements as well
        for (const auto& c : space)
          if (c.vec == 4) cand.push_back({8, c.ept, c.waves, c.grid_mult, c.tile_r, c.tile_c});
    } else if (policy == 2) {
      if (!cm) fail(COOT_EINVAL, "the MLP policy needs a cost model");
      if (is_dim_kind(mode)) fail(COOT_EUNSUPPORTED, "the cost model covers element-wise evaluation and accu");
      int64_t R, C;
      infer_shape(*h->e, operands, &R, &C);
      // rank only the configurations these operands allow (alignment, tile)
      std::vector<int32_t> ok(space.size());
      st = coot_tune_runnable(h, operands, out, mode, dim, space.data(), (uint32_t)space.size(), ok.data());
      if (st != COOT_OK) fail(st, last_error());
      std::vector<coot_launch_cfg> live;
      for (size_t i = 0; i < space.size(); ++i)
        if (ok[i]) live.push_back(space[i]);
      uint32_t bi = 0;
      std::vector<float> pred(live.size());
      st = coot_costmodel_predict(cm, h, R, C, mode < 0 ? 0 : 1, live.data(), (uint32_t)live.size(), pred.data(), &bi,
                                  stream);
      if (st != COOT_OK) fail(st, last_error());
      // Leave the library default only for a predicted gain of kCostModelMargin or more
      // (predictions are log times): where the network sees no clear winner, the default,
      // chosen from the same kind of timing tables, is as likely to be right.
      const coot_launch_cfg d = library_default();
      for (size_t i = 0; i < live.size(); ++i)
        if (std::memcmp(&live[i], &d, sizeof d) == 0 && pred[bi] > pred[i] - std::log(1.0f + kCostModelMargin))
          bi = (uint32_t)i;
      cand.push_back(live[bi]);
    } else {
      fail(COOT_EINVAL, "policy must be 0, 1 or 2");
    }
    std::vector<float> t(cand.size());
    st = coot_tune_table(h, operands, scalars, out, mode, dim, cand.data(), (uint32_t)cand.size(), 5, 0, t.data(),
                         stream);
    if (st != COOT_OK) fail(st, last_error());
    size_t bi = 0;
    for (size_t i = 0; i < t.size(); ++i)
      if (!std::isnan(t[i]) && (std::isnan(t[bi]) || t[i] < t[bi])) bi = i;
    if (policy == 1 && !std::isnan(t[bi])) {
      // Medians of 5 rounds separate configurations only to a few per cent: the
      // finalists (within 5 % of the fastest, at most 4) are timed again side by side
      // over 21 interleaved rounds, and the fastest of those is kept.
      std::vector<size_t> fin;
      for (size_t i = 0; i < t.size(); ++i)
        if (!std::isnan(t[i]) && t[i] <= 1.05f * t[bi]) fin.push_back(i);
      std::sort(fin.begin(), fin.end(), [&](size_t x, size_t y) { return t[x] < t[y]; });
      if (fin.size() > 4) fin.resize(4);
      if (fin.size() > 1) {
        std::vector<coot_launch_cfg> fc;
        for (size_t i : fin) fc.push_back(cand[i]);
        std::vector<float> ft(fc.size());
        st = coot_tune_table(h, operands, scalars, out, mode, dim, fc.data(), (uint32_t)fc.size(), 21, 0, ft.data(),
                             stream);
        if (st != COOT_OK) fail(st, last_error());
        size_t fb = 0;
        for (size_t i = 0; i < ft.size(); ++i)
          if (!std::isnan(ft[i]) && (std::isnan(ft[fb]) || ft[i] < ft[fb])) fb = i;
        if (!std::isnan(ft[fb])) {
          bi = fin[fb];
          t[bi] = ft[fb];
          // Finalists the repeated-call timing cannot tell apart (within 2 %) are
          // told apart by one launch after a cache flush (operands from HBM): the
          // kept configuration then also suits callers whose operands are not cached.
          std::vector<size_t> tie;
          for (size_t i = 0; i < ft.size(); ++i)
            if (!std::isnan(ft[i]) && ft[i] <= 1.02f * ft[fb]) tie.push_back(i);
          if (tie.size() > 1) {
            std::vector<coot_launch_cfg> tc;
            for (size_t i : tie) tc.push_back(fc[i]);
            std::vector<float> ct(tc.size());
            st = coot_tune_table(h, operands, scalars, out, mode, dim, tc.data(), (uint32_t)tc.size(), 5, 1,
                                 ct.data(), stream);
            if (st != COOT_OK) fail(st, last_error());
            size_t cb = 0;
            for (size_t i = 0; i < ct.size(); ++i)
              if (!std::isnan(ct[i]) && (std::isnan(ct[cb]) || ct[i] < ct[cb])) cb = i;
            if (!std::isnan(ct[cb])) {
              bi = fin[tie[cb]];
              t[bi] = ft[tie[cb]];
            }
          }
        }
      }
    }
    *best = cand[bi];
    if (best_us) *best_us = t[bi];
  });
}

}  // extern "C"
