// C boundary of the contact-surrogate MLP (include/vmas.h): the handle owns
// the FP32 master parameters, the Adam moments, the BF16 copies in the
// kernels' layouts and the training workspace.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "vmas.h"
#include "vmas_internal.h"

namespace vmas {
int mlp_nparam();
int64_t mlp_parts_for(int64_t n);
hipError_t mlp_launch_forward(const unsigned short* W1, const unsigned short* W2,
                              const unsigned short* W3, const float* b1, const float* b2,
                              const float* b3, const float* X, int64_t n, const int32_t* n_dev,
                              const int32_t* out_idx, float* Y, float* H1, float* H2,
                              hipStream_t s);
hipError_t mlp_launch_backward(const unsigned short* W1, const unsigned short* W2,
                               const unsigned short* W3, const float* b1, const float* b2,
                               const float* b3, const float* X, const float* H1, const float* H2,
                               const float* dY, int64_t n, float* dX, float* part, float* grad,
                               hipStream_t s);
hipError_t mlp_launch_mse(const float* Y, const float* tgt, int64_t n, float* dY, float* row_loss,
                          hipStream_t s);
hipError_t mlp_launch_adam(float* master, float* mom, float* var, const float* grad, float lr,
                           float b1, float b2, float eps, int step, unsigned short* W1,
                           unsigned short* W2, unsigned short* W3, float* bias1, float* bias2,
                           float* bias3, hipStream_t s);
hipError_t mlp_launch_unpack(const float* master, unsigned short* W1, unsigned short* W2,
                             unsigned short* W3, float* bias1, float* bias2, float* bias3,
                             hipStream_t s);
hipError_t mlp_launch_sum(const float* v, int64_t n, float* out, hipStream_t s);
vmas_status set_error(vmas_status st, const char* fmt, ...);
}  // namespace vmas

using namespace vmas;

struct vmas_mlp {
  int device = 0;
  int step = 0;
  float* master = nullptr;  // [NP] fp32
  float* mom = nullptr;
  float* var = nullptr;
  float* grad = nullptr;
  unsigned short *W1 = nullptr, *W2 = nullptr, *W3 = nullptr;  // bf16, padded
  float *b1 = nullptr, *b2 = nullptr, *b3 = nullptr;
  // workspace
  int64_t cap = 0;
  float *H1 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *rl = nullptr, *part = nullptr;
};

namespace {

constexpr int NH = 128, NIP = 16, NOP = 16;

#define MCHK(expr) \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return set_error(VMAS_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(d);
  }
  ~Dev() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void free_ws(vmas_mlp* m) {
  float* ps[] = {m->H1, m->H2, m->Y, m->dY, m->rl, m->part};
  for (float* p : ps)
    if (p) (void)hipFree(p);
  m->H1 = m->H2 = m->Y = m->dY = m->rl = m->part = nullptr;
  m->cap = 0;
}

vmas_status ensure_ws(vmas_mlp* m, int64_t n) {
  if (n <= m->cap) return VMAS_OK;
  free_ws(m);
  const size_t P = (size_t)mlp_parts_for(n) * mlp_nparam();
  hipError_t e = hipSuccess;
  if ((e = hipMalloc((void**)&m->H1, n * NH * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&m->H2, n * NH * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&m->Y, n * 2 * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&m->dY, n * 2 * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&m->rl, n * sizeof(float))) != hipSuccess ||
      (e = hipMalloc((void**)&m->part, P * sizeof(float))) != hipSuccess) {
    free_ws(m);
    return set_error(VMAS_ERR_OUT_OF_MEMORY, "MLP workspace for %lld rows: %s", (long long)n,
                     hipGetErrorString(e));
  }
  m->cap = n;
  return VMAS_OK;
}

void free_mlp(vmas_mlp* m) {
  if (!m) return;
  free_ws(m);
  void* ps[] = {m->master, m->mom, m->var, m->grad, m->W1, m->W2, m->W3, m->b1, m->b2, m->b3};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

}  // namespace

extern "C" {

int32_t vmas_mlp_num_params(void) { return mlp_nparam(); }

vmas_status vmas_mlp_create(const float* params, uint64_t seed, int device, vmas_mlp** out) {
  if (!out) return set_error(VMAS_ERR_INVALID_ARGUMENT, "out must not be NULL");
  *out = nullptr;
  const int NP = mlp_nparam();
  std::vector<float> host(NP);
  if (params) {
    for (int i = 0; i < NP; ++i) {
      if (!std::isfinite(params[i]))
        return set_error(VMAS_ERR_INVALID_ARGUMENT, "params[%d] is not finite", i);
      host[i] = params[i];
    }
  } else {
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer, canonical order
    std::mt19937_64 rng(seed);
    const int sizes[6] = {NH * 12, NH, NH * NH, NH, 2 * NH, 2};
    const int fans[6] = {12, 12, NH, NH, NH, NH};
    int o = 0;
    for (int k = 0; k < 6; ++k) {
      std::uniform_real_distribution<float> u(-1.0f / std::sqrt((float)fans[k]),
                                              1.0f / std::sqrt((float)fans[k]));
      for (int i = 0; i < sizes[k]; ++i) host[o++] = u(rng);
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return set_error(VMAS_ERR_DEVICE, "no HIP device is available");
  if (device < 0 || device >= ndev)
    return set_error(VMAS_ERR_INVALID_ARGUMENT, "device %d outside [0, %d)", device, ndev);
  Dev g(device);
  vmas_mlp* m = new vmas_mlp();
  m->device = device;
  hipError_t e = hipSuccess;
  const size_t fb = NP * sizeof(float);
  if ((e = hipMalloc((void**)&m->master, fb)) != hipSuccess || (e = hipMalloc((void**)&m->mom, fb)) != hipSuccess ||
      (e = hipMalloc((void**)&m->var, fb)) != hipSuccess || (e = hipMalloc((void**)&m->grad, fb)) != hipSuccess ||
      (e = hipMalloc((void**)&m->W1, NH * NIP * 2)) != hipSuccess ||
      (e = hipMalloc((void**)&m->W2, NH * NH * 2)) != hipSuccess ||
      (e = hipMalloc((void**)&m->W3, NOP * NH * 2)) != hipSuccess ||
      (e = hipMalloc((void**)&m->b1, NH * 4)) != hipSuccess || (e = hipMalloc((void**)&m->b2, NH * 4)) != hipSuccess ||
      (e = hipMalloc((void**)&m->b3, 2 * 4)) != hipSuccess) {
    free_mlp(m);
    return set_error(VMAS_ERR_OUT_OF_MEMORY, "MLP parameters: %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpy(m->master, host.data(), fb, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(m->mom, 0, fb)) != hipSuccess || (e = hipMemset(m->var, 0, fb)) != hipSuccess ||
      (e = hipMemset(m->W1, 0, NH * NIP * 2)) != hipSuccess ||
      (e = hipMemset(m->W3, 0, NOP * NH * 2)) != hipSuccess ||
      (e = mlp_launch_unpack(m->master, m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, nullptr)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    free_mlp(m);
    return set_error(VMAS_ERR_DEVICE, "MLP upload: %s", hipGetErrorString(e));
  }
  *out = m;
  return VMAS_OK;
}

vmas_status vmas_mlp_destroy(vmas_mlp* m) {
  if (!m) return VMAS_OK;
  Dev g(m->device);
  free_mlp(m);
  return VMAS_OK;
}

vmas_status vmas_mlp_get_params(const vmas_mlp* m, float* out, void* stream) {
  if (!m || !out) return set_error(VMAS_ERR_INVALID_ARGUMENT, "mlp and out must not be NULL");
  Dev g(m->device);
  MCHK(hipMemcpyAsync(out, m->master, mlp_nparam() * sizeof(float), hipMemcpyDeviceToHost,
                      (hipStream_t)stream));
  MCHK(hipStreamSynchronize((hipStream_t)stream));
  return VMAS_OK;
}

vmas_status vmas_mlp_forward(vmas_mlp* m, const float* X, int64_t n, float* Y, void* stream) {
  if (!m || (n > 0 && (!X || !Y))) return set_error(VMAS_ERR_INVALID_ARGUMENT, "mlp, X and Y are required");
  if (n < 0) return set_error(VMAS_ERR_INVALID_ARGUMENT, "n must be >= 0");
  Dev g(m->device);
  MCHK(mlp_launch_forward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, n, nullptr, nullptr, Y, nullptr, nullptr,
                          (hipStream_t)stream));
  return VMAS_OK;
}


vmas_status vmas_mlp_backward(vmas_mlp* m, const float* X, int64_t n, const float* dY,
                              float* grad, float* dX, void* stream) {
  if (!m || (n > 0 && (!X || !dY))) return set_error(VMAS_ERR_INVALID_ARGUMENT, "mlp, X and dY are required");
  if (n < 1) return set_error(VMAS_ERR_INVALID_ARGUMENT, "n must be >= 1");
  Dev g(m->device);
  vmas_status st = ensure_ws(m, n);
  if (st != VMAS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  MCHK(mlp_launch_forward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, n, nullptr, nullptr, m->Y, m->H1, m->H2, s));
  MCHK(mlp_launch_backward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, m->H1, m->H2, dY, n, dX,
                           m->part, grad ? grad : m->grad, s));
  return VMAS_OK;
}

vmas_status vmas_mlp_train_step(vmas_mlp* m, const float* X, const float* target, int64_t n,
                                float lr, float* loss, void* stream) {
  if (!m || !X || !target) return set_error(VMAS_ERR_INVALID_ARGUMENT, "mlp, X and target are required");
  if (n < 1) return set_error(VMAS_ERR_INVALID_ARGUMENT, "n must be >= 1");
  if (!(std::isfinite(lr) && lr >= 0)) return set_error(VMAS_ERR_INVALID_ARGUMENT, "lr must be finite and >= 0");
  Dev g(m->device);
  vmas_status st = ensure_ws(m, n);
  if (st != VMAS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  MCHK(mlp_launch_forward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, n, nullptr, nullptr, m->Y, m->H1, m->H2, s));
  MCHK(mlp_launch_mse(m->Y, target, n, m->dY, m->rl, s));
  if (loss) MCHK(mlp_launch_sum(m->rl, n, loss, s));
  MCHK(mlp_launch_backward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, m->H1, m->H2, m->dY, n,
                           nullptr, m->part, m->grad, s));
  m->step += 1;
  MCHK(mlp_launch_adam(m->master, m->mom, m->var, m->grad, lr, 0.9f, 0.999f, 1e-8f, m->step, m->W1,
                       m->W2, m->W3, m->b1, m->b2, m->b3, s));
  return VMAS_OK;
}

}  // extern "C"

namespace vmas {
// Forward over min(max_n, *d_n) rows, the count read on the device (rows
// compacted by a preceding kernel on the same stream); row r's output goes
// to Y[out_idx[r]] when out_idx is given.
vmas_status mlp_forward_counted(vmas_mlp* m, const float* X, int64_t max_n, const int32_t* d_n,
                                const int32_t* out_idx, float* Y, hipStream_t s) {
  Dev g(m->device);
  MCHK(mlp_launch_forward(m->W1, m->W2, m->W3, m->b1, m->b2, m->b3, X, max_n, d_n, out_idx, Y,
                          nullptr, nullptr, s));
  return VMAS_OK;
}
}  // namespace vmas
