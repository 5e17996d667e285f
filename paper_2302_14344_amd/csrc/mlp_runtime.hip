// Host side of the warm-start network: the subadmm_mlp_* entry points of
// include/subadmm.h.  Layout of the bound workspace (256-byte aligned sub-arrays):
// FP32 master parameters, gradients and the two Adam moments; BF16 copies of the
// weights; per layer the BF16 input activations of the last forward batch; the FP32
// output; two FP32 gradient buffers; split-K and column-sum partials.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/subadmm.h"
#include "mlp_internal.hpp"

#define SUBADMM_API extern "C" __attribute__((visibility("default")))

using namespace subadmm;

namespace {
constexpr int kSplits = 16;      // split-K factor of the weight gradients
constexpr int kColSplits = 64;   // row chunks of the bias-gradient column sums
constexpr int kLossBlocks = 1024;
thread_local std::string g_mlp_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

struct subadmm_mlp {
  int32_t L = 0, max_batch = 0, max_w = 0;
  std::vector<int32_t> w;          // widths
  std::vector<int64_t> off_W, off_b, off_Wbf, off_act;  // element offsets
  int64_t P = 0, n_wbf = 0, n_act = 0, max_wk = 0;
  struct {
    size_t P, G, M, V, Wbf, act, y, dz0, dz1, part, cpart, lpart, aff, total;
  } o{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  bool affine = false;
  uint64_t gen = 0;  // advanced on bind and on input-affine changes
  int32_t last_batch = -1;
  std::string err;
};

namespace {

int mfail(subadmm_mlp* m, int code, const std::string& msg) {
  if (m) m->err = msg;
  else g_mlp_error = msg;
  return code;
}

int mdev(subadmm_mlp* m, hipError_t e, const char* where) {
  if (e == hipSuccess) return SUBADMM_OK;
  return mfail(m, SUBADMM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename X>
X* mat(subadmm_mlp* m, size_t off) {
  return reinterpret_cast<X*>(m->ws + off);
}

}  // namespace

SUBADMM_API int subadmm_mlp_create(int32_t n_layers, const int32_t* widths, int32_t max_batch, subadmm_mlp** out) {
  if (!out) return mfail(nullptr, SUBADMM_E_ARG, "out is null");
  *out = nullptr;
  if (n_layers < 1 || n_layers > 16 || !widths) return mfail(nullptr, SUBADMM_E_ARG, "bad layer count");
  if (max_batch < 1 || max_batch > (1 << 24)) return mfail(nullptr, SUBADMM_E_ARG, "bad max_batch");
  auto* m = new subadmm_mlp();
  m->L = n_layers;
  m->max_batch = max_batch;
  for (int32_t k = 0; k <= n_layers; ++k) {
    if (widths[k] < 1 || widths[k] > 1024) {
      delete m;
      return mfail(nullptr, SUBADMM_E_ARG, "widths must be in 1..1024");
    }
    m->w.push_back(widths[k]);
    m->max_w = std::max(m->max_w, widths[k]);
  }
  int64_t p = 0, wb = 0, ac = 0;
  for (int32_t k = 0; k < n_layers; ++k) {
    const int64_t nk = m->w[k + 1], kk = m->w[k];
    m->off_W.push_back(p);
    p += nk * kk;
    m->off_b.push_back(p);
    p += nk;
    m->off_Wbf.push_back(wb);
    wb += nk * kk;
    m->off_act.push_back(ac);
    ac += (int64_t)max_batch * kk;
    m->max_wk = std::max(m->max_wk, nk * kk);
  }
  m->P = p;
  m->n_wbf = wb;
  m->n_act = ac;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + (bytes ? bytes : 1));
    return o;
  };
  const size_t fb = sizeof(float);
  m->o.P = take(fb * m->P);
  m->o.G = take(fb * m->P);
  m->o.M = take(fb * m->P);
  m->o.V = take(fb * m->P);
  m->o.Wbf = take(2 * (size_t)m->n_wbf);
  m->o.act = take(2 * (size_t)m->n_act);
  m->o.y = take(fb * (size_t)max_batch * m->w[n_layers]);
  m->o.dz0 = take(fb * (size_t)max_batch * m->max_w);
  m->o.dz1 = take(fb * (size_t)max_batch * m->max_w);
  m->o.part = take(fb * (size_t)kSplits * m->max_wk);
  m->o.cpart = take(fb * (size_t)kColSplits * m->max_w);
  m->o.lpart = take(sizeof(double) * kLossBlocks);
  m->o.aff = take(fb * 2 * (size_t)m->w[0]);
  m->o.total = off;
  *out = m;
  return SUBADMM_OK;
}

SUBADMM_API int64_t subadmm_mlp_param_count(const subadmm_mlp* m) { return m ? m->P : 0; }
SUBADMM_API size_t subadmm_mlp_workspace_bytes(const subadmm_mlp* m) { return m ? m->o.total : 0; }

SUBADMM_API int subadmm_mlp_bind(subadmm_mlp* m, void* dev_workspace, size_t bytes, void* hip_stream) {
  if (!m) return mfail(nullptr, SUBADMM_E_ARG, "null network");
  if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255))
    return mfail(m, SUBADMM_E_ARG, "workspace must be non-null and 256-byte aligned");
  if (bytes < m->o.total) return mfail(m, SUBADMM_E_WORKSPACE, "workspace too small");
  m->ws = static_cast<char*>(dev_workspace);
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->bound = true;
  m->affine = false;
  ++m->gen;
  m->last_batch = -1;
  return mdev(m, hipMemsetAsync(m->ws, 0, m->o.total, m->stream), "mlp bind clear");
}

namespace {

int refresh_bf16(subadmm_mlp* m) {
  for (int32_t k = 0; k < m->L; ++k) {
    const int rc = mdev(m, launch_cast_bf16(mat<float>(m, m->o.P) + m->off_W[k], mat<uint16_t>(m, m->o.Wbf) + m->off_Wbf[k],
                                            (long)m->w[k + 1] * m->w[k], m->stream),
                        "cast weights");
    if (rc) return rc;
  }
  return SUBADMM_OK;
}

int check_bound(subadmm_mlp* m) {
  if (!m) return mfail(nullptr, SUBADMM_E_ARG, "null network");
  if (!m->bound) return mfail(m, SUBADMM_E_WORKSPACE, "network has no bound workspace");
  return SUBADMM_OK;
}

}  // namespace

SUBADMM_API int subadmm_mlp_set_params(subadmm_mlp* m, const float* params) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (!params) return mfail(m, SUBADMM_E_ARG, "null params");
  hipError_t e = hipMemcpyAsync(m->ws + m->o.P, params, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->ws + m->o.M, 0, sizeof(float) * m->P, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->ws + m->o.V, 0, sizeof(float) * m->P, m->stream);
  rc = mdev(m, e, "set params");
  if (rc) return rc;
  return refresh_bf16(m);
}

SUBADMM_API int subadmm_mlp_set_input_affine(subadmm_mlp* m, const float* scale, const float* shift) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (!scale != !shift) return mfail(m, SUBADMM_E_ARG, "scale and shift must both be set or both be null");
  if (!scale) {
    m->affine = false;
    ++m->gen;
    return SUBADMM_OK;
  }
  const size_t bytes = sizeof(float) * m->w[0];
  hipError_t e = hipMemcpyAsync(m->ws + m->o.aff, scale, bytes, hipMemcpyDeviceToDevice, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->ws + m->o.aff + bytes, shift, bytes, hipMemcpyDeviceToDevice, m->stream);
  rc = mdev(m, e, "set input affine");
  if (!rc) m->affine = true;
  ++m->gen;
  return rc;
}

SUBADMM_API int subadmm_mlp_get_params(subadmm_mlp* m, float* params_out) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (!params_out) return mfail(m, SUBADMM_E_ARG, "null output");
  return mdev(m, hipMemcpyAsync(params_out, m->ws + m->o.P, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream),
              "get params");
}

SUBADMM_API int subadmm_mlp_forward(subadmm_mlp* m, int32_t batch, const float* x, float* y) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (batch < 0 || batch > m->max_batch) return mfail(m, SUBADMM_E_ARG, "batch out of range");
  if (!x || !y) return mfail(m, SUBADMM_E_ARG, "null input/output");
  m->last_batch = batch;
  if (batch == 0) return SUBADMM_OK;
  uint16_t* act = mat<uint16_t>(m, m->o.act);
  const uint16_t* Wb = mat<uint16_t>(m, m->o.Wbf);
  const float* P = mat<float>(m, m->o.P);
  float* ybuf = mat<float>(m, m->o.y);
  if (m->affine) {
    const float* aff = mat<float>(m, m->o.aff);
    rc = mdev(m, launch_cast_affine_bf16(x, aff, aff + m->w[0], m->w[0], act + m->off_act[0], (long)batch * m->w[0],
                                         m->stream),
              "normalise input");
  } else {
    rc = mdev(m, launch_cast_bf16(x, act + m->off_act[0], (long)batch * m->w[0], m->stream), "cast input");
  }
  if (rc) return rc;
  for (int32_t k = 0; k < m->L; ++k) {
    const long N = m->w[k + 1], K = m->w[k];
    GemmArgs<uint16_t, uint16_t> g{};
    g.A = act + m->off_act[k];
    g.sam = K;
    g.sak = 1;
    g.B = Wb + m->off_Wbf[k];
    g.sbk = 1;
    g.sbn = K;
    g.M = batch;
    g.N = N;
    g.K = K;
    g.k_chunk = (K + 31) / 32 * 32;
    g.a_m_fast = 0;
    g.b_n_fast = 0;
    g.bias = P + m->off_b[k];
    if (k + 1 < m->L) {
      g.epi = EPI_BIAS_RELU_BF16;
      g.out_bf16 = act + m->off_act[k + 1];
      g.ldo = N;
    } else {
      g.epi = EPI_BIAS_F32;
      g.C = ybuf;
      g.ldc = N;
    }
    rc = mdev(m, launch_gemm(g, 1, m->stream), "forward gemm");
    if (rc) return rc;
  }
  return mdev(m, hipMemcpyAsync(y, ybuf, sizeof(float) * (size_t)batch * m->w[m->L], hipMemcpyDeviceToDevice, m->stream),
              "copy output");
}

SUBADMM_API int subadmm_mlp_backward(subadmm_mlp* m, int32_t batch, const float* target, const float* wt,
                                     float* grad_out, float* loss_out) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (batch != m->last_batch) return mfail(m, SUBADMM_E_STATE, "backward needs the batch of the last forward");
  if (!target) return mfail(m, SUBADMM_E_ARG, "null target");
  float* G = mat<float>(m, m->o.G);
  if (batch == 0) {
    rc = mdev(m, hipMemsetAsync(G, 0, sizeof(float) * m->P, m->stream), "clear grad");
    if (rc) return rc;
  } else {
    const uint16_t* act = mat<uint16_t>(m, m->o.act);
    const uint16_t* Wb = mat<uint16_t>(m, m->o.Wbf);
    float* dz[2] = {mat<float>(m, m->o.dz0), mat<float>(m, m->o.dz1)};
    float* part = mat<float>(m, m->o.part);
    float* cpart = mat<float>(m, m->o.cpart);
    float* lossp = loss_out;
    rc = mdev(m, launch_loss_grad(mat<float>(m, m->o.y), target, wt, dz[0], (long)batch * m->w[m->L],
                                  mat<double>(m, m->o.lpart), kLossBlocks, lossp, m->stream),
              "loss gradient");
    if (rc) return rc;
    int cur = 0;
    for (int32_t k = m->L - 1; k >= 0; --k) {
      const long N = m->w[k + 1], K = m->w[k];
      // dW_k = dZ^T A_k (split over the batch, partials summed in a fixed order)
      GemmArgs<float, uint16_t> gw{};
      gw.A = dz[cur];
      gw.sam = 1;
      gw.sak = N;
      gw.B = act + m->off_act[k];
      gw.sbk = K;
      gw.sbn = 1;
      gw.M = N;
      gw.N = K;
      gw.K = batch;
      const long per = ((long)batch + kSplits - 1) / kSplits;
      gw.k_chunk = (per + 31) / 32 * 32;
      const int splits = (int)(((long)batch + gw.k_chunk - 1) / gw.k_chunk);
      gw.a_m_fast = 1;
      gw.b_n_fast = 1;
      gw.epi = EPI_STORE;
      gw.C = part;
      gw.ldc = K;
      gw.c_split = N * K;
      rc = mdev(m, launch_gemm(gw, splits, m->stream), "weight gradient gemm");
      if (!rc) rc = mdev(m, launch_sum_partials(part, splits, N * K, G + m->off_W[k], m->stream), "weight gradient sum");
      if (!rc) rc = mdev(m, launch_colsum(dz[cur], batch, (int)N, cpart, kColSplits, G + m->off_b[k], m->stream),
                         "bias gradient");
      if (rc) return rc;
      if (k > 0) {
        // dA_k = dZ W_k, through the ReLU that produced A_k
        GemmArgs<float, uint16_t> ga{};
        ga.A = dz[cur];
        ga.sam = N;
        ga.sak = 1;
        ga.B = Wb + m->off_Wbf[k];
        ga.sbk = K;
        ga.sbn = 1;
        ga.M = batch;
        ga.N = K;
        ga.K = N;
        ga.k_chunk = (N + 31) / 32 * 32;
        ga.a_m_fast = 0;
        ga.b_n_fast = 1;
        ga.epi = EPI_RELU_MASK;
        ga.mask = act + m->off_act[k];
        ga.ldm = K;
        ga.C = dz[1 - cur];
        ga.ldc = K;
        rc = mdev(m, launch_gemm(ga, 1, m->stream), "input gradient gemm");
        if (rc) return rc;
        cur = 1 - cur;
      }
    }
  }
  if (grad_out)
    return mdev(m, hipMemcpyAsync(grad_out, G, sizeof(float) * m->P, hipMemcpyDeviceToDevice, m->stream), "copy grad");
  return SUBADMM_OK;
}

SUBADMM_API int subadmm_mlp_adam(subadmm_mlp* m, float lr, float beta1, float beta2, float eps, int32_t step) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return mfail(m, SUBADMM_E_ARG, "bad Adam hyper-parameters");
  rc = mdev(m, launch_adam(mat<float>(m, m->o.P), mat<float>(m, m->o.G), mat<float>(m, m->o.M), mat<float>(m, m->o.V),
                           (long)m->P, lr, beta1, beta2, eps, step, m->stream),
            "adam");
  if (rc) return rc;
  return refresh_bf16(m);
}

SUBADMM_API int subadmm_mlp_gather_rows(subadmm_mlp* m, const float* src, int64_t n_rows, int32_t width,
                                        const int32_t* idx, int32_t count, float* dst) {
  int rc = check_bound(m);
  if (rc) return rc;
  if (n_rows < 0 || width < 1 || count < 0) return mfail(m, SUBADMM_E_ARG, "bad gather sizes");
  if (count > 0 && (!src || !idx || !dst)) return mfail(m, SUBADMM_E_ARG, "null array");
  return mdev(m, launch_gather_rows(src, (long)n_rows, width, idx, count, dst, m->stream), "gather rows");
}

SUBADMM_API void subadmm_mlp_destroy(subadmm_mlp* m) { delete m; }

int32_t mlp_input_width(const subadmm_mlp* m) { return m->w.front(); }
int32_t mlp_output_width(const subadmm_mlp* m) { return m->w.back(); }
int32_t mlp_max_batch(const subadmm_mlp* m) { return m->max_batch; }
hipStream_t mlp_stream(const subadmm_mlp* m) { return m->stream; }
uint64_t mlp_generation(const subadmm_mlp* m) { return m->gen; }

int mlp_infer_on(subadmm_mlp* m, hipStream_t s, int32_t batch, const float* x, float* y) {
  bool fits = m->L <= kInferMaxLayers;
  for (int32_t k = 0; k <= m->L && fits; ++k) fits = m->w[k] <= kInferMaxWidth;
  if (!fits) return mlp_forward_on(m, s, batch, x, y);
  int rc = check_bound(m);
  if (rc) return rc;
  if (batch < 0 || batch > m->max_batch) return mfail(m, SUBADMM_E_ARG, "batch out of range");
  if (!x || !y) return mfail(m, SUBADMM_E_ARG, "null input/output");
  m->last_batch = -1;  // no activations kept: a backward pass needs a forward first
  MlpInferArgs a{};
  a.x = x;
  a.y = y;
  if (m->affine) {
    a.scale = mat<float>(m, m->o.aff);
    a.shift = a.scale + m->w[0];
  }
  a.Wbf = mat<uint16_t>(m, m->o.Wbf);
  a.P = mat<float>(m, m->o.P);
  a.batch = batch;
  a.L = m->L;
  for (int32_t k = 0; k <= m->L; ++k) a.w[k] = m->w[k];
  for (int32_t k = 0; k < m->L; ++k) {
    a.off_Wbf[k] = (long)m->off_Wbf[k];
    a.off_b[k] = (long)m->off_b[k];
    a.vec_w[k] = (m->w[k] % 8 == 0 && m->off_Wbf[k] % 8 == 0) ? 1 : 0;
  }
  return mdev(m, launch_mlp_infer(a, s), "inference");
}

SUBADMM_API int subadmm_mlp_infer(subadmm_mlp* m, int32_t batch, const float* x, float* y) {
  if (!m) return SUBADMM_E_ARG;
  return mlp_infer_on(m, m->stream, batch, x, y);
}

int mlp_forward_on(subadmm_mlp* m, hipStream_t s, int32_t batch, const float* x, float* y) {
  const hipStream_t own = m->stream;
  m->stream = s;
  const int rc = subadmm_mlp_forward(m, batch, x, y);
  m->stream = own;
  return rc;
}

SUBADMM_API const char* subadmm_mlp_last_error(const subadmm_mlp* m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }
