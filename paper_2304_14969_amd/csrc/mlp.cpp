// Host side of the separability-proposal network: parameter storage on the
// device, forward passes for scoring, gradients and Adam training, all run by
// the kernels of k_mlp.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mlp.h"
#include "qs_internal.h"

namespace qs {
void* device_alloc(size_t bytes);
void device_free(void* p);
void set_last_error(const char* msg);
}  // namespace qs

namespace {

constexpr int kScoreRowsFloats = qs::kScoreRows * (QS_MLP_INPUTS + 1);

int mfail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  qs::set_last_error(buf);
  return code;
}

int merr(hipError_t e, const char* what) {
  if (e == hipSuccess) return QS_OK;
  return mfail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Scratch for `rows` rows: X, y, z, H1, H2, D3, D2, D1, L.
struct Scratch {
  float *X = nullptr, *y = nullptr, *z = nullptr, *H1 = nullptr, *H2 = nullptr, *D3 = nullptr,
        *D2 = nullptr, *D1 = nullptr, *L = nullptr;
  void* block = nullptr;
  bool alloc(uint64_t rows) {
    const size_t f = rows * (QS_MLP_INPUTS + 1 + 1 + 64 + 64 + 1 + 64 + 64 + 1);
    block = qs::device_alloc(f * sizeof(float));
    if (!block) return false;
    float* p = static_cast<float*>(block);
    X = p; p += rows * QS_MLP_INPUTS;
    y = p; p += rows;
    z = p; p += rows;
    H1 = p; p += rows * 64;
    H2 = p; p += rows * 64;
    D3 = p; p += rows;
    D2 = p; p += rows * 64;
    D1 = p; p += rows * 64;
    L = p;
    return true;
  }
  ~Scratch() { qs::device_free(block); }
};

}  // namespace

namespace qs {

// scores[r] = sigmoid(logit) of the rows of host X (rows x 32); synchronizes.
int mlp_scores(qs_mlp* net, const float* X, uint64_t rows, float* scores) {
  if (rows == 0) return QS_OK;
  if (rows <= uint64_t(kScoreRows)) {
    // the usual case (the dirty qubits of one separation round): the kernel
    // reads the rows from and writes the logits to mapped pinned memory
    float* hz = net->hscore + kScoreRows * QS_MLP_INPUTS;
    float* dz = net->dscore + kScoreRows * QS_MLP_INPUTS;
    std::memcpy(net->hscore, X, rows * QS_MLP_INPUTS * sizeof(float));
    hipError_t e = launch_mlp_score(net->P, net->dscore, int(rows), dz, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (int rc = merr(e, "network forward")) return rc;
    for (uint64_t r = 0; r < rows; ++r) scores[r] = 1.0f / (1.0f + std::exp(-hz[r]));
    return QS_OK;
  }
  Scratch s;
  if (!s.alloc(rows)) return mfail(QS_E_NOMEM, "network scratch");
  hipError_t e = hipMemcpyAsync(s.X, X, rows * QS_MLP_INPUTS * sizeof(float), hipMemcpyHostToDevice,
                                net->stream);
  if (e == hipSuccess)
    e = launch_mlp_forward(net->P, s.X, int(rows), s.z, nullptr, nullptr, net->stream);
  std::vector<float> z(rows);
  if (e == hipSuccess)
    e = hipMemcpyAsync(z.data(), s.z, rows * sizeof(float), hipMemcpyDeviceToHost, net->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
  if (int rc = merr(e, "network forward")) return rc;
  for (uint64_t r = 0; r < rows; ++r) scores[r] = 1.0f / (1.0f + std::exp(-z[r]));
  return QS_OK;
}

}  // namespace qs

extern "C" {

int qs_mlp_create(qs_mlp** out) {
  if (!out) return mfail(QS_E_INVAL, "out is NULL");
  qs_mlp* n = new qs_mlp();
  const int np = qs::mlp_param_count();
  void* blk = qs::device_alloc(size_t(4) * np * sizeof(float));
  if (!blk) {
    delete n;
    return mfail(QS_E_NOMEM, "network parameters");
  }
  const size_t score_floats = size_t(kScoreRowsFloats);
  if (hipHostMalloc(reinterpret_cast<void**>(&n->hscore), score_floats * sizeof(float),
                    hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&n->dscore), n->hscore, 0) != hipSuccess) {
    if (n->hscore) (void)hipHostFree(n->hscore);
    qs::device_free(blk);
    delete n;
    return mfail(QS_E_NOMEM, "network scoring buffers");
  }
  n->block = blk;
  n->P = static_cast<float*>(blk);
  n->M = n->P + np;
  n->V = n->M + np;
  n->G = n->V + np;
  std::vector<float> zero(size_t(4) * np, 0.0f);
  hipError_t e = hipMemcpy(blk, zero.data(), zero.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipHostFree(n->hscore);
    qs::device_free(blk);
    delete n;
    return merr(e, "network init");
  }
  *out = n;
  return QS_OK;
}

int qs_mlp_free(qs_mlp* n) {
  if (!n) return QS_OK;
  (void)hipStreamSynchronize(n->stream);
  qs::device_free(n->block);
  (void)hipHostFree(n->hscore);
  delete n;
  return QS_OK;
}

int qs_mlp_set_stream(qs_mlp* n, void* stream) {
  if (!n) return mfail(QS_E_INVAL, "network is NULL");
  n->stream = static_cast<hipStream_t>(stream);
  return QS_OK;
}

int qs_mlp_set_params(qs_mlp* n, const float* host, uint64_t count) {
  if (!n || !host) return mfail(QS_E_INVAL, "NULL argument");
  if (count != uint64_t(QS_MLP_PARAMS)) return mfail(QS_E_INVAL, "expected %d parameters", QS_MLP_PARAMS);
  for (uint64_t i = 0; i < count; ++i)
    if (!std::isfinite(host[i])) return mfail(QS_E_INVAL, "parameter %llu is not finite", (unsigned long long)i);
  hipError_t e = hipMemcpyAsync(n->P, host, count * sizeof(float), hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return merr(e, "set params");
}

int qs_mlp_get_params(qs_mlp* n, float* host, uint64_t count) {
  if (!n || !host) return mfail(QS_E_INVAL, "NULL argument");
  if (count != uint64_t(QS_MLP_PARAMS)) return mfail(QS_E_INVAL, "expected %d parameters", QS_MLP_PARAMS);
  hipError_t e = hipMemcpyAsync(host, n->P, count * sizeof(float), hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return merr(e, "get params");
}

int qs_mlp_forward(qs_mlp* n, const float* X, uint64_t rows, float* scores) {
  if (!n || (rows && (!X || !scores))) return mfail(QS_E_INVAL, "NULL argument");
  if (rows > (uint64_t(1) << 30)) return mfail(QS_E_INVAL, "too many rows");
  return qs::mlp_scores(n, X, rows, scores);
}

int qs_mlp_grad(qs_mlp* n, const float* X, const float* y, uint64_t rows, float* grad,
                double* loss) {
  if (!n || !X || !y || !grad) return mfail(QS_E_INVAL, "NULL argument");
  if (rows == 0 || rows > (uint64_t(1) << 24)) return mfail(QS_E_INVAL, "rows = %llu", (unsigned long long)rows);
  Scratch s;
  if (!s.alloc(rows)) return mfail(QS_E_NOMEM, "network scratch");
  hipError_t e = hipMemcpyAsync(s.X, X, rows * QS_MLP_INPUTS * sizeof(float), hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s.y, y, rows * sizeof(float), hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = qs::launch_mlp_forward(n->P, s.X, int(rows), s.z, s.H1, s.H2, n->stream);
  if (e == hipSuccess)
    e = qs::launch_mlp_backward(n->P, s.X, s.y, int(rows), s.z, s.H1, s.H2, s.D3, s.D2, s.D1, s.L, n->G, n->stream);
  std::vector<float> L(rows);
  if (e == hipSuccess)
    e = hipMemcpyAsync(grad, n->G, QS_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(L.data(), s.L, rows * sizeof(float), hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (int rc = merr(e, "network gradient")) return rc;
  if (loss) {
    double t = 0.0;
    for (float v : L) t += v;
    *loss = t / double(rows);
  }
  return QS_OK;
}

int qs_mlp_train(qs_mlp* n, const float* X, const float* y, uint64_t rows, const qs_train_cfg* cfg,
                 double* final_loss) {
  if (!n || !X || !y || !cfg) return mfail(QS_E_INVAL, "NULL argument");
  if (rows == 0 || rows > (uint64_t(1) << 26)) return mfail(QS_E_INVAL, "rows = %llu", (unsigned long long)rows);
  const uint64_t B = cfg->batch ? cfg->batch : 256;
  if (B > rows) return mfail(QS_E_INVAL, "batch larger than the data");
  if (!(cfg->lr > 0) || !(cfg->beta1 >= 0 && cfg->beta1 < 1) || !(cfg->beta2 >= 0 && cfg->beta2 < 1))
    return mfail(QS_E_INVAL, "bad optimizer settings");
  // the whole data set on the device, minibatches are consecutive rows
  Scratch data, mb;
  if (!data.alloc(rows) || !mb.alloc(B)) return mfail(QS_E_NOMEM, "training buffers");
  hipError_t e = hipMemcpyAsync(data.X, X, rows * QS_MLP_INPUTS * sizeof(float), hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(data.y, y, rows * sizeof(float), hipMemcpyHostToDevice, n->stream);
  // fresh optimizer moments
  if (e == hipSuccess)
    e = hipMemsetAsync(n->M, 0, size_t(2) * QS_MLP_PARAMS * sizeof(float), n->stream);
  double b1t = 1.0, b2t = 1.0;
  uint64_t cursor = 0;
  for (uint32_t step = 1; step <= cfg->steps && e == hipSuccess; ++step) {
    if (cursor + B > rows) cursor = 0;
    const float* Xb = data.X + cursor * QS_MLP_INPUTS;
    const float* yb = data.y + cursor;
    cursor += B;
    e = qs::launch_mlp_forward(n->P, Xb, int(B), mb.z, mb.H1, mb.H2, n->stream);
    if (e == hipSuccess)
      e = qs::launch_mlp_backward(n->P, Xb, yb, int(B), mb.z, mb.H1, mb.H2, mb.D3, mb.D2, mb.D1, mb.L, n->G, n->stream);
    b1t *= cfg->beta1;
    b2t *= cfg->beta2;
    if (e == hipSuccess)
      e = qs::launch_mlp_adam(n->P, n->M, n->V, n->G, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps,
                              float(1.0 / (1.0 - b1t)), float(1.0 / (1.0 - b2t)), n->stream);
  }
  if (e == hipSuccess && final_loss) {
    // mean loss over the whole data set with the trained parameters
    e = qs::launch_mlp_forward(n->P, data.X, int(rows), data.z, data.H1, data.H2, n->stream);
    if (e == hipSuccess)
      e = qs::launch_mlp_backward(n->P, data.X, data.y, int(rows), data.z, data.H1, data.H2, data.D3,
                                  data.D2, data.D1, data.L, n->G, n->stream);
    std::vector<float> L(rows);
    if (e == hipSuccess) e = hipMemcpyAsync(L.data(), data.L, rows * sizeof(float), hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    double t = 0.0;
    for (float v : L) t += v;
    *final_loss = t / double(rows);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return merr(e, "network training");
}

}  // extern "C"
