// Host runtime of the warm-start MLP (k_mlp.hip): parameters, activations and gradients on
// the device; a training step is forward, loss, back-propagation and (optionally) Adam, all
// launched on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace elmfb;

static thread_local std::string g_mlp_error;

struct elmfb_mlp_s {
  int L = 0, max_batch = 0, max_dim = 0, n_mod = 1;
  std::vector<int> dims;
  std::vector<int64_t> offW, offb;
  int64_t n_params = 0;
  int64_t t = 0;                         // Adam steps taken
  std::string err;
  std::vector<void*> allocs;
  float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr, *d_y = nullptr;
  uint16_t *d_pb = nullptr, *d_x = nullptr, *d_g1 = nullptr, *d_g2 = nullptr;
  std::vector<uint16_t*> d_act;          // a_l, l = 1..L-1 (bfloat16)
  double *d_part = nullptr, *d_loss = nullptr;
  float* d_ws = nullptr;                 // split-k partial products of the weight gradients
  float* d_colpart = nullptr;            // partial column sums of the bias gradients
};

namespace {

constexpr int kLossParts = 1024;

elmfb_status mfail(elmfb_mlp m, elmfb_status code, const std::string& msg) {
  if (m) m->err = msg;
  g_mlp_error = msg;
  return code;
}

#define MHIP(m, expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return mfail((m), ELMFB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t malloc_track(elmfb_mlp m, T** p, int64_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)(bytes > 0 ? bytes : 16));
  if (e != hipSuccess) return e;
  m->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

void release(elmfb_mlp m) {
  for (void* p : m->allocs) hipFree(p);
  m->allocs.clear();
}

// z = a W^T + b over a batch: A = activations [batch][n_in] (row-major), B(k, n) = W[n][k]
MlpGemm layer_gemm(elmfb_mlp m, int l, const uint16_t* a_in, int batch) {
  MlpGemm g{};
  g.M = batch;
  g.N = m->dims[l + 1];
  g.K = m->dims[l];
  g.A = a_in;
  g.sam = m->dims[l];
  g.sak = 1;
  g.B = m->d_pb + m->offW[l];
  g.sbk = 1;
  g.sbn = m->dims[l];
  g.bias = m->d_p + m->offb[l];
  g.ldo = m->dims[l + 1];
  return g;
}

hipError_t run_forward(elmfb_mlp m, const float* x, int batch, float* y, hipStream_t s) {
  hipError_t e = launch_mlp_to_bf16((int64_t)batch * m->dims[0], x, m->d_x, s);
  const uint16_t* a = m->d_x;
  for (int l = 0; l < m->L && e == hipSuccess; ++l) {
    MlpGemm g = layer_gemm(m, l, a, batch);
    if (l < m->L - 1) {
      g.epi = MLP_EPI_BIAS_TANH;
      g.out_bf16 = m->d_act[l + 1];
      a = m->d_act[l + 1];
    } else {
      g.epi = MLP_EPI_BIAS;
      g.out_f32 = y;
    }
    e = launch_mlp_gemm(g, nullptr, s);
  }
  return e;
}

}  // namespace

extern "C" {

elmfb_status elmfb_mlp_create(int32_t n_layers, const int32_t* dims_host, int32_t n_mod,
                              int32_t max_batch, elmfb_mlp* out) {
  if (!out || !dims_host) return mfail(nullptr, ELMFB_E_INVALID, "NULL argument");
  *out = nullptr;
  if (n_layers < 1 || n_layers > 16) return mfail(nullptr, ELMFB_E_INVALID, "n_layers must be in 1..16");
  if (max_batch < 1 || max_batch > (1 << 24))
    return mfail(nullptr, ELMFB_E_INVALID, "max_batch must be in 1..2^24");
  for (int l = 0; l <= n_layers; ++l)
    if (dims_host[l] < 1 || dims_host[l] > 65536)
      return mfail(nullptr, ELMFB_E_INVALID, "layer widths must be in 1..65536");
  if (n_mod < 1 || n_mod > 64 || dims_host[n_layers] % n_mod != 0)
    return mfail(nullptr, ELMFB_E_INVALID, "n_mod must be in 1..64 and divide the output width");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return mfail(nullptr, ELMFB_E_DEVICE, "no HIP device available");
  elmfb_mlp m = new (std::nothrow) elmfb_mlp_s();
  if (!m) return mfail(nullptr, ELMFB_E_NOMEM, "host allocation failed");
  m->L = n_layers;
  m->n_mod = n_mod;
  m->max_batch = max_batch;
  m->dims.assign(dims_host, dims_host + n_layers + 1);
  int64_t o = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->offW.push_back(o);
    o += (int64_t)m->dims[l] * m->dims[l + 1];
    m->offb.push_back(o);
    o += m->dims[l + 1];
  }
  m->n_params = o;
  for (int d : m->dims) m->max_dim = std::max(m->max_dim, d);
  const int64_t B = max_batch;
  hipError_t e = hipSuccess;
  auto A = [&](auto** p, int64_t bytes) {
    if (e == hipSuccess) e = malloc_track(m, p, bytes);
  };
  A(&m->d_p, o * 4);
  A(&m->d_g, o * 4);
  A(&m->d_m, o * 4);
  A(&m->d_v, o * 4);
  A(&m->d_pb, o * 2);
  A(&m->d_x, B * m->dims[0] * 2);
  A(&m->d_y, B * m->dims[n_layers] * 4);
  A(&m->d_g1, B * m->max_dim * 2);
  A(&m->d_g2, B * m->max_dim * 2);
  m->d_act.assign(n_layers + 1, nullptr);
  for (int l = 1; l < n_layers; ++l) A(&m->d_act[l], B * m->dims[l] * 2);
  A(&m->d_part, kLossParts * 8);
  A(&m->d_loss, 8);
  int64_t ws = 0;
  for (int l = 0; l < n_layers; ++l)
    ws = std::max(ws, mlp_gemm_ws_floats(m->dims[l + 1], m->dims[l], max_batch));
  A(&m->d_ws, ws * 4);
  A(&m->d_colpart, (int64_t)mlp_colsum_chunks(max_batch) * m->max_dim * 4);
  if (e == hipSuccess) e = hipMemset(m->d_p, 0, (size_t)o * 4);
  if (e == hipSuccess) e = hipMemset(m->d_pb, 0, (size_t)o * 2);
  if (e == hipSuccess) e = hipMemset(m->d_m, 0, (size_t)o * 4);
  if (e == hipSuccess) e = hipMemset(m->d_v, 0, (size_t)o * 4);
  if (e != hipSuccess) {
    const std::string msg = std::string("MLP allocation: ") + hipGetErrorString(e);
    release(m);
    delete m;
    return mfail(nullptr, ELMFB_E_NOMEM, msg);
  }
  *out = m;
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_query(elmfb_mlp m, int64_t* n_params) {
  if (!m || !n_params) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  *n_params = m->n_params;
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_set_params(elmfb_mlp m, const float* params_host) {
  if (!m || !params_host) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  for (int64_t i = 0; i < m->n_params; ++i)
    if (!std::isfinite(params_host[i])) return mfail(m, ELMFB_E_NUMERIC, "non-finite parameter");
  MHIP(m, hipMemcpy(m->d_p, params_host, (size_t)m->n_params * 4, hipMemcpyHostToDevice));
  MHIP(m, launch_mlp_to_bf16(m->n_params, m->d_p, m->d_pb, nullptr));
  MHIP(m, hipMemset(m->d_m, 0, (size_t)m->n_params * 4));
  MHIP(m, hipMemset(m->d_v, 0, (size_t)m->n_params * 4));
  MHIP(m, hipDeviceSynchronize());
  m->t = 0;
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_get_params(elmfb_mlp m, float* params_host) {
  if (!m || !params_host) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  MHIP(m, hipDeviceSynchronize());
  MHIP(m, hipMemcpy(params_host, m->d_p, (size_t)m->n_params * 4, hipMemcpyDeviceToHost));
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_get_grads(elmfb_mlp m, float* grads_host) {
  if (!m || !grads_host) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  MHIP(m, hipDeviceSynchronize());
  MHIP(m, hipMemcpy(grads_host, m->d_g, (size_t)m->n_params * 4, hipMemcpyDeviceToHost));
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_forward(elmfb_mlp m, const float* x_dev, const float* f_dev,
                               int32_t batch, float* y_dev, void* stream) {
  if (!m || !x_dev || !y_dev) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  if (m->n_mod > 1 && !f_dev) return mfail(m, ELMFB_E_INVALID, "modulated network needs f");
  if (batch < 1 || batch > m->max_batch) return mfail(m, ELMFB_E_INVALID, "batch out of range");
  hipStream_t s = (hipStream_t)stream;
  if (m->n_mod == 1) {
    MHIP(m, run_forward(m, x_dev, batch, y_dev, s));
  } else {
    const int K = m->dims[m->L] / m->n_mod;
    MHIP(m, run_forward(m, x_dev, batch, m->d_y, s));
    MHIP(m, launch_mlp_modulate((int64_t)batch * K, K, m->n_mod, m->d_y, f_dev, y_dev, s));
  }
  return ELMFB_OK;
}

elmfb_status elmfb_mlp_train_step(elmfb_mlp m, const float* x_dev, const float* f_dev,
                                  const float* t_dev, int32_t batch, const elmfb_adam* opt,
                                  double* loss_host, void* stream) {
  if (!m || !x_dev || !t_dev) return mfail(m, ELMFB_E_INVALID, "NULL argument");
  if (m->n_mod > 1 && !f_dev) return mfail(m, ELMFB_E_INVALID, "modulated network needs f");
  if (batch < 1 || batch > m->max_batch) return mfail(m, ELMFB_E_INVALID, "batch out of range");
  if (opt && !(opt->lr > 0.0 && opt->beta1 >= 0.0 && opt->beta1 < 1.0 && opt->beta2 >= 0.0 &&
               opt->beta2 < 1.0 && opt->eps > 0.0))
    return mfail(m, ELMFB_E_INVALID, "bad Adam settings");
  hipStream_t s = (hipStream_t)stream;
  const int L = m->L;
  MHIP(m, run_forward(m, x_dev, batch, m->d_y, s));
  if (m->n_mod == 1) {
    MHIP(m, launch_mlp_loss((int64_t)batch * m->dims[L], m->d_y, t_dev, m->d_g1, m->d_part,
                            kLossParts, m->d_loss, s));
  } else {
    const int K = m->dims[L] / m->n_mod;
    MHIP(m, launch_mlp_mod_loss((int64_t)batch * K, K, m->n_mod, m->d_y, f_dev, t_dev, m->d_g1,
                                m->d_part, kLossParts, m->d_loss, s));
  }
  uint16_t* g = m->d_g1;
  uint16_t* g_next = m->d_g2;
  for (int l = L - 1; l >= 0; --l) {
    const int n_in = m->dims[l], n_out = m->dims[l + 1];
    const uint16_t* a_in = l == 0 ? m->d_x : m->d_act[l];
    // dW_l[n][k] = sum_m g[m][n] a_in[m][k]
    MlpGemm gw{};
    gw.M = n_out;
    gw.N = n_in;
    gw.K = batch;
    gw.A = g;
    gw.sam = 1;
    gw.sak = n_out;
    gw.B = a_in;
    gw.sbk = n_in;
    gw.sbn = 1;
    gw.epi = MLP_EPI_F32;
    gw.out_f32 = m->d_g + m->offW[l];
    gw.ldo = n_in;
    MHIP(m, launch_mlp_gemm(gw, m->d_ws, s));
    MHIP(m, launch_mlp_colsum(batch, n_out, g, m->d_colpart, m->d_g + m->offb[l], s));
    if (l > 0) {
      // g_prev[m][k] = (sum_n g[m][n] W[n][k]) (1 - a_in[m][k]^2)
      MlpGemm gb{};
      gb.M = batch;
      gb.N = n_in;
      gb.K = n_out;
      gb.A = g;
      gb.sam = n_out;
      gb.sak = 1;
      gb.B = m->d_pb + m->offW[l];
      gb.sbk = n_in;
      gb.sbn = 1;
      gb.epi = MLP_EPI_DTANH;
      gb.act = a_in;
      gb.out_bf16 = g_next;
      gb.ldo = n_in;
      MHIP(m, launch_mlp_gemm(gb, nullptr, s));
      std::swap(g, g_next);
    }
  }
  if (opt) {
    m->t += 1;
    const double c1 = 1.0 - std::pow(opt->beta1, (double)m->t);
    const double c2 = 1.0 - std::pow(opt->beta2, (double)m->t);
    MHIP(m, launch_mlp_adam(m->n_params, m->d_p, m->d_g, m->d_m, m->d_v, m->d_pb, (float)opt->lr,
                            (float)opt->beta1, (float)opt->beta2, (float)opt->eps, (float)c1,
                            (float)c2, s));
  }
  if (loss_host) {
    MHIP(m, hipMemcpyAsync(loss_host, m->d_loss, 8, hipMemcpyDeviceToHost, s));
    MHIP(m, hipStreamSynchronize(s));
  }
  return ELMFB_OK;
}

void elmfb_mlp_destroy(elmfb_mlp m) {
  if (!m) return;
  hipDeviceSynchronize();
  release(m);
  delete m;
}

const char* elmfb_mlp_last_error(elmfb_mlp m) {
  if (m) return m->err.c_str();
  return g_mlp_error.c_str();
}

}  // extern "C"
