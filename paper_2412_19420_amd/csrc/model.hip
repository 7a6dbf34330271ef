// Host side of the scheduler's cost model (bm_model_*): creation, training on
// the device with the hand-written forward/backward/Adam kernels, prediction,
// persistence.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "handles.hpp"
#include "mlp.hpp"

namespace bm {

namespace {

// splitmix64: counter-based generator (Steele, Lea, Flood 2014).
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

double uniform01(uint64_t seed, uint64_t i) {
  return (double)(splitmix64(seed * 0x100000001B3ull + i) >> 11) * (1.0 / 9007199254740992.0);
}

const char kMagic[8] = {'B', 'M', 'M', 'L', 'P', '0', '0', '1'};

struct DevData {
  const float* p = nullptr;
  DBuf<float> own;
};

// Device view of a host or device float array of n elements.
DevData as_device(const float* src, uint64_t n, hipStream_t s) {
  DevData d;
  if (is_device_ptr(src)) {
    d.p = src;
  } else {
    d.own.reset(n, s);
    BM_HIP(hipMemcpyAsync(d.own.get(), src, n * 4, hipMemcpyHostToDevice, s));
    BM_HIP(hipStreamSynchronize(s));
    d.p = d.own.get();
  }
  return d;
}

std::vector<float> to_host(const float* src, uint64_t n) {
  std::vector<float> h(n);
  if (n == 0) return h;
  if (is_device_ptr(src)) BM_HIP(hipMemcpy(h.data(), src, n * 4, hipMemcpyDeviceToHost));
  else std::memcpy(h.data(), src, n * 4);
  return h;
}

void upload_norm(bm_model* m, hipStream_t s) {
  BM_HIP(hipMemcpyAsync(m->norm.get(), m->h_norm, sizeof(m->h_norm), hipMemcpyHostToDevice, s));
  BM_HIP(hipStreamSynchronize(s));
}

}  // namespace

bm_model* model_create(uint32_t seed) {
  std::unique_ptr<bm_model> m(new bm_model);
  BM_HIP(hipGetDevice(&m->device));
  hipStream_t s = nullptr;
  m->master.reset(MLP_PARAMS, s);
  m->m.reset(MLP_PARAMS, s);
  m->v.reset(MLP_PARAMS, s);
  m->grad.reset(MLP_PARAMS, s);
  m->wbf.reset(MLP_PARAMS, s);
  m->norm.reset(2 * MLP_IN, s);
  // He-uniform weights, zero biases
  std::vector<float> w(MLP_PARAMS, 0.f);
  auto init = [&](int off, int fan_in, int count) {
    const double lim = std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) w[off + i] = (float)((2.0 * uniform01(seed, off + i) - 1.0) * lim);
  };
  init(MLP_W1, MLP_IN, MLP_IN * MLP_H);
  init(MLP_W2, MLP_H, MLP_H * MLP_H);
  init(MLP_W3, MLP_H, MLP_H);
  BM_HIP(hipMemcpy(m->master.get(), w.data(), MLP_PARAMS * 4, hipMemcpyHostToDevice));
  launch_fill_u32(reinterpret_cast<uint32_t*>(m->m.get()), 0, MLP_PARAMS, s);
  launch_fill_u32(reinterpret_cast<uint32_t*>(m->v.get()), 0, MLP_PARAMS, s);
  for (int i = 0; i < MLP_IN; ++i) {
    m->h_norm[i] = 0.f;
    m->h_norm[MLP_IN + i] = 1.f;
  }
  upload_norm(m.get(), s);
  launch_mlp_round(m->master.get(), m->wbf.get(), s);
  BM_HIP(hipStreamSynchronize(s));
  return m.release();
}

void model_set_norm_from(bm_model* m, const float* feats, uint64_t rows, hipStream_t s) {
  std::vector<float> h = to_host(feats, rows * MLP_IN);
  for (int i = 0; i < MLP_IN; ++i) {
    double sum = 0, sq = 0;
    for (uint64_t r = 0; r < rows; ++r) sum += h[r * MLP_IN + i];
    const double mean = rows ? sum / rows : 0.0;
    for (uint64_t r = 0; r < rows; ++r) {
      const double d = h[r * MLP_IN + i] - mean;
      sq += d * d;
    }
    const double sd = rows > 1 ? std::sqrt(sq / (rows - 1)) : 0.0;
    m->h_norm[i] = (float)mean;
    m->h_norm[MLP_IN + i] = sd > 1e-6 ? (float)(1.0 / sd) : 1.f;
  }
  m->has_norm = true;
  upload_norm(m, s);
}

std::vector<float> model_train(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                               uint32_t epochs, float lr, uint32_t batch, bool graph,
                               hipStream_t caller) {
  if (rows == 0 || epochs == 0) return {};
  if (!m->has_norm) model_set_norm_from(m, feats, rows, caller);
  if (batch == 0) batch = 256;
  // training runs on a private stream (a graph cannot be captured on the null
  // stream), ordered after the caller's stream
  hipStream_t ts = nullptr;
  hipEvent_t ev = nullptr;
  BM_HIP(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking));
  struct Cleanup {
    hipStream_t s;
    hipEvent_t e;
    ~Cleanup() {
      if (e) (void)hipEventDestroy(e);
      if (s) (void)hipStreamDestroy(s);
    }
  } cleanup{ts, nullptr};
  BM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  cleanup.e = ev;
  BM_HIP(hipEventRecord(ev, caller));
  BM_HIP(hipStreamWaitEvent(ts, ev, 0));
  DevData X = as_device(feats, rows * MLP_IN, ts);
  DevData Y = as_device(labels, rows, ts);
  const uint32_t nb = (uint32_t)((rows + batch - 1) / batch);
  DBuf<float> partial((uint64_t)mlp_grad_slots(std::min<uint64_t>(batch, rows)) * (MLP_PARAMS + 1), ts);
  DBuf<float> acc(1, ts), losses(epochs, ts);
  DBuf<uint32_t> ctr(2, ts);  // [0] epoch, [1] Adam steps taken before this epoch
  launch_fill_u32(reinterpret_cast<uint32_t*>(acc.get()), 0, 1, ts);
  launch_fill_u32(ctr.get(), 0, 1, ts);
  launch_fill_u32(ctr.get() + 1, (uint32_t)m->step, 1, ts);
  auto epoch = [&] {
    for (uint32_t b = 0; b < nb; ++b) {
      const uint64_t r0 = (uint64_t)b * batch, r1 = std::min<uint64_t>(rows, r0 + batch);
      launch_mlp_grad(X.p, Y.p, r0, r1, 1.f / (float)(r1 - r0), m->wbf.get(), m->norm.get(),
                      partial.get(), m->grad.get(), acc.get(), ts);
      launch_mlp_adam(m->master.get(), m->m.get(), m->v.get(), m->grad.get(), m->wbf.get(), lr,
                      ctr.get() + 1, b + 1, ts);
    }
    launch_mlp_epoch_end(acc.get(), losses.get(), ctr.get(), nb, ts);
  };
  if (graph && epochs > 1) {
    // one epoch is 2 * batches + 1 small launches: capture it once, replay it
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    BM_HIP(hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal));
    try {
      epoch();
    } catch (...) {
      (void)hipStreamEndCapture(ts, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    BM_HIP(hipStreamEndCapture(ts, &g));
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BM_HIP(e);
    for (uint32_t i = 0; i < epochs && e == hipSuccess; ++i) e = hipGraphLaunch(ge, ts);
    (void)hipGraphExecDestroy(ge);
    BM_HIP(e);
  } else {
    for (uint32_t i = 0; i < epochs; ++i) epoch();
  }
  std::vector<float> out(epochs);
  BM_HIP(hipMemcpyAsync(out.data(), losses.get(), epochs * 4, hipMemcpyDeviceToHost, ts));
  BM_HIP(hipStreamSynchronize(ts));
  m->step += (uint64_t)nb * epochs;
  return out;
}

void model_predict(const bm_model* m, const float* feats, uint64_t rows, float* out,
                   hipStream_t s) {
  if (rows == 0) return;
  DevData X = as_device(feats, rows * MLP_IN, s);
  if (is_device_ptr(out)) {
    launch_mlp_forward(X.p, rows, m->wbf.get(), m->norm.get(), out, s);
  } else {
    DBuf<float> o(rows, s);
    launch_mlp_forward(X.p, rows, m->wbf.get(), m->norm.get(), o.get(), s);
    BM_HIP(hipMemcpyAsync(out, o.get(), rows * 4, hipMemcpyDeviceToHost, s));
  }
  BM_HIP(hipStreamSynchronize(s));
}

void model_predict_device(const bm_model* m, const float* dfeats, uint64_t rows, float* dout,
                          hipStream_t s) {
  launch_mlp_forward(dfeats, rows, m->wbf.get(), m->norm.get(), dout, s);
}

float model_grad(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                 float* grad_out, hipStream_t s) {
  DevData X = as_device(feats, rows * MLP_IN, s);
  DevData Y = as_device(labels, rows, s);
  DBuf<float> loss(1, s);
  launch_fill_u32(reinterpret_cast<uint32_t*>(loss.get()), 0, 1, s);
  if (rows) {
    DBuf<float> partial((uint64_t)mlp_grad_slots(rows) * (MLP_PARAMS + 1), s);
    launch_mlp_grad(X.p, Y.p, 0, rows, 1.f / (float)rows, m->wbf.get(), m->norm.get(), partial.get(),
                    m->grad.get(), loss.get(), s);
    BM_HIP(hipStreamSynchronize(s));
  } else {
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->grad.get()), 0, MLP_PARAMS, s);
  }
  float l = 0.f;
  BM_HIP(hipMemcpyAsync(&l, loss.get(), 4, hipMemcpyDeviceToHost, s));
  if (grad_out)
    BM_HIP(hipMemcpyAsync(grad_out, m->grad.get(), MLP_PARAMS * 4, hipMemcpyDefault, s));
  BM_HIP(hipStreamSynchronize(s));
  return l;
}

void model_params(const bm_model* m, float* master, float* rounded, float* norm) {
  if (master) BM_HIP(hipMemcpy(master, m->master.get(), MLP_PARAMS * 4, hipMemcpyDefault));
  if (rounded) {
    std::vector<uint16_t> h(MLP_PARAMS);
    BM_HIP(hipMemcpy(h.data(), m->wbf.get(), MLP_PARAMS * 2, hipMemcpyDeviceToHost));
    for (int i = 0; i < MLP_PARAMS; ++i) {
      const uint32_t u = (uint32_t)h[i] << 16;
      std::memcpy(&rounded[i], &u, 4);
    }
  }
  if (norm) std::memcpy(norm, m->h_norm, sizeof(m->h_norm));
}

void model_set_params(bm_model* m, const float* master, const float* norm) {
  hipStream_t s = nullptr;
  if (master) {
    BM_HIP(hipMemcpy(m->master.get(), master, MLP_PARAMS * 4, hipMemcpyDefault));
    launch_mlp_round(m->master.get(), m->wbf.get(), s);
  }
  if (norm) {
    std::memcpy(m->h_norm, norm, sizeof(m->h_norm));
    m->has_norm = true;
    upload_norm(m, s);
  }
  BM_HIP(hipStreamSynchronize(s));
}

void model_save(const bm_model* m, const char* path) {
  std::vector<float> w(MLP_PARAMS);
  BM_HIP(hipMemcpy(w.data(), m->master.get(), MLP_PARAMS * 4, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) fail(BM_ERR_INVALID_ARG, "cannot open %s for writing", path);
  const uint32_t n = MLP_PARAMS, hn = m->has_norm ? 1u : 0u;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 &&
            std::fwrite(&hn, 4, 1, f) == 1 && std::fwrite(m->h_norm, 4, 2 * MLP_IN, f) == 2 * MLP_IN &&
            std::fwrite(w.data(), 4, MLP_PARAMS, f) == (size_t)MLP_PARAMS;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) fail(BM_ERR_INVALID_ARG, "write to %s failed", path);
}

bm_model* model_load(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) fail(BM_ERR_INVALID_ARG, "cannot open %s", path);
  char mg[8];
  uint32_t n = 0, hn = 0;
  float norm[2 * MLP_IN];
  std::vector<float> w(MLP_PARAMS);
  const bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0 &&
                  std::fread(&n, 4, 1, f) == 1 && n == (uint32_t)MLP_PARAMS &&
                  std::fread(&hn, 4, 1, f) == 1 && std::fread(norm, 4, 2 * MLP_IN, f) == 2 * MLP_IN &&
                  std::fread(w.data(), 4, MLP_PARAMS, f) == (size_t)MLP_PARAMS;
  std::fclose(f);
  if (!ok) fail(BM_ERR_INVALID_ARG, "%s is not a cost-model file", path);
  std::unique_ptr<bm_model> m(model_create(0));
  model_set_params(m.get(), w.data(), norm);
  m->has_norm = hn != 0;
  return m.release();
}

}  // namespace bm
