// Host side of the learned-closure network: lbm_mlp objects, training steps,
// column moments.  The lattice-facing calls live in lbm_api.cpp.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lbm_internal.h"

namespace {

#define MTRY(call)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      char m_[256];                                                                           \
      snprintf(m_, sizeof m_, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return lbm::set_error(e_ == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, m_);       \
    }                                                                                         \
  } while (0)

constexpr int64_t kMaxBatch = 65536;

}  // namespace

struct lbm_mlp {
  hipStream_t stream = nullptr;
  float* master = nullptr;  // FP32 weights
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  uint16_t* Wb = nullptr;   // bfloat16 copies, padded layouts
  float* gpart = nullptr;   // per-block gradients [blocks][params]
  double* lpart = nullptr;  // per-block squared errors
  float* grad = nullptr;    // reduced gradient
  double* loss = nullptr;
  float* norm = nullptr;    // optional z-score (mean[36], 1/std[36], out scale[3])
  int use_norm = 0;
  float noise = 0.0f;       // training input noise (z-scored units)
  uint64_t seed = 0;
  int step = 0;
};

namespace lbm {
MlpDevice mlp_device(const lbm_mlp* m) { return MlpDevice{m->Wb, m->master}; }
}  // namespace lbm

namespace {

void free_mlp(lbm_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  (void)hipFree(m->master);
  (void)hipFree(m->m);
  (void)hipFree(m->v);
  (void)hipFree(m->Wb);
  (void)hipFree(m->gpart);
  (void)hipFree(m->lpart);
  (void)hipFree(m->grad);
  (void)hipFree(m->loss);
  (void)hipFree(m->norm);
  delete m;
}

// Refreshes the bfloat16 copies from the master weights (no update).
lbm_status refresh(lbm_mlp* m) {
  MTRY(lbm::launch_mlp_adam(m->gpart, 0, m->lpart, m->master, m->m, m->v, m->Wb, nullptr, nullptr, 0, 0.0f,
                            0.0, m->stream));
  return LBM_OK;
}

lbm_status create_impl(lbm_mlp* m, const float* init) {
  const size_t np = lbm::kMlpParams * sizeof(float);
  MTRY(hipMalloc(&m->master, np));
  MTRY(hipMalloc(&m->m, np));
  MTRY(hipMalloc(&m->v, np));
  MTRY(hipMalloc(&m->grad, np));
  MTRY(hipMalloc(&m->Wb, lbm::kMlpBf16 * sizeof(uint16_t)));
  MTRY(hipMalloc(&m->gpart, (size_t)lbm::mlp_blocks(kMaxBatch) * np));
  MTRY(hipMalloc(&m->lpart, (size_t)lbm::mlp_blocks(kMaxBatch) * sizeof(double)));
  MTRY(hipMalloc(&m->loss, sizeof(double)));
  MTRY(hipMalloc(&m->norm, sizeof(float) * lbm::kClosureNorm));
  MTRY(hipMemsetAsync(m->m, 0, np, m->stream));
  MTRY(hipMemsetAsync(m->v, 0, np, m->stream));
  // padding of the bfloat16 layouts must be zero
  MTRY(hipMemsetAsync(m->Wb, 0, lbm::kMlpBf16 * sizeof(uint16_t), m->stream));
  if (init)
    MTRY(hipMemcpyAsync(m->master, init, np, hipMemcpyHostToDevice, m->stream));
  else
    MTRY(hipMemsetAsync(m->master, 0, np, m->stream));
  lbm_status st = refresh(m);
  if (st != LBM_OK) return st;
  MTRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_mlp_create(const float* init, void* stream, lbm_mlp** out) {
  if (!out) return lbm::set_error(LBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  lbm_mlp* m = new lbm_mlp();
  m->stream = (hipStream_t)stream;
  lbm_status st = create_impl(m, init);
  if (st != LBM_OK) {
    free_mlp(m);
    return st;
  }
  *out = m;
  return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m) { free_mlp(m); }

lbm_status lbm_mlp_get_params(lbm_mlp* m, float* out) {
  if (!m || !out) return lbm::set_error(LBM_ERR_INVALID_ARG, "NULL argument");
  MTRY(hipStreamSynchronize(m->stream));
  MTRY(hipMemcpy(out, m->master, lbm::kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_mlp_set_params(lbm_mlp* m, const float* in) {
  if (!m || !in) return lbm::set_error(LBM_ERR_INVALID_ARG, "NULL argument");
  MTRY(hipMemcpyAsync(m->master, in, lbm::kMlpParams * sizeof(float), hipMemcpyHostToDevice, m->stream));
  lbm_status st = refresh(m);
  if (st != LBM_OK) return st;
  MTRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_set_norm(lbm_mlp* m, const float* norm) {
  if (!m) return lbm::set_error(LBM_ERR_INVALID_ARG, "NULL network");
  if (norm) MTRY(hipMemcpyAsync(m->norm, norm, sizeof(float) * lbm::kClosureNorm, hipMemcpyHostToDevice, m->stream));
  MTRY(hipStreamSynchronize(m->stream));
  m->use_norm = norm ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_mlp_set_noise(lbm_mlp* m, float amplitude, uint64_t seed) {
  if (!m || !(amplitude >= 0.0f)) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad noise arguments");
  m->noise = amplitude;
  m->seed = seed;
  return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp* m, const float* x, int64_t M, float* y) {
  if (!m || !x || !y || M < 0 || M > (int64_t)1 << 30) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad forward arguments");
  if (M == 0) return LBM_OK;
  MTRY(lbm::launch_mlp_forward(x, (int)M, m->Wb, m->master, m->use_norm ? m->norm : nullptr, y, m->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_train_step(lbm_mlp* m, const float* x, const float* t, const int32_t* idx, int64_t B,
                              float lr, double* loss) {
  if (!m || !x || !t || B < 1 || B > kMaxBatch || !(lr >= 0.0f))
    return lbm::set_error(LBM_ERR_INVALID_ARG, "bad train-step arguments");
  MTRY(lbm::launch_mlp_train(x, t, idx, (int)B, m->Wb, m->master, m->use_norm ? m->norm : nullptr, m->gpart,
                              m->lpart, m->noise, m->seed * 0x100000001B3ull + (uint64_t)m->step, m->stream));
  m->step += 1;
  MTRY(lbm::launch_mlp_adam(m->gpart, lbm::mlp_blocks(B), m->lpart, m->master, m->m, m->v, m->Wb, nullptr,
                            m->loss, m->step, lr, 1.0 / (3.0 * (double)B), m->stream));
  if (loss) {
    MTRY(hipStreamSynchronize(m->stream));
    MTRY(hipMemcpy(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost));
  }
  return LBM_OK;
}

lbm_status lbm_mlp_gradient(lbm_mlp* m, const float* x, const float* t, int64_t B, float* grad, double* loss) {
  if (!m || !x || !t || !grad || B < 1 || B > kMaxBatch)
    return lbm::set_error(LBM_ERR_INVALID_ARG, "bad gradient arguments");
  MTRY(lbm::launch_mlp_train(x, t, nullptr, (int)B, m->Wb, m->master, m->use_norm ? m->norm : nullptr, m->gpart,
                              m->lpart, 0.0f, 0, m->stream));
  MTRY(lbm::launch_mlp_adam(m->gpart, lbm::mlp_blocks(B), m->lpart, m->master, m->m, m->v, m->Wb, m->grad,
                            m->loss, 0, 0.0f, 1.0 / (3.0 * (double)B), m->stream));
  MTRY(hipStreamSynchronize(m->stream));
  MTRY(hipMemcpy(grad, m->grad, lbm::kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
  if (loss) MTRY(hipMemcpy(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_column_moments(const float* x, int64_t M, int32_t ncols, double* mean, double* std, void* stream) {
  if (!x || M < 1 || ncols < 1 || ncols > 65536 || !mean || !std)
    return lbm::set_error(LBM_ERR_INVALID_ARG, "bad moments arguments");
  double* d = nullptr;
  MTRY(hipMalloc(&d, sizeof(double) * 2 * ncols));
  std::vector<double> h(2 * (size_t)ncols);
  hipError_t e = lbm::launch_column_moments(x, M, ncols, d, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(h.data(), d, sizeof(double) * 2 * ncols, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  for (int c = 0; c < ncols; ++c) {
    const double a = h[c] / (double)M, b = h[ncols + c] / (double)M;
    mean[c] = a;
    std[c] = std::sqrt(std::max(0.0, b - a * a));
  }
  return LBM_OK;
}

}  // extern "C"
