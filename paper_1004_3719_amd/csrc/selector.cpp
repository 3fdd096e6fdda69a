// Learned per-block format selection: the model object, its file format, the
// build-time inference hook, block features and the per-block timing harness.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "host.h"
#include "launch.h"
#include "mlp.h"

struct ffx_selector_s {
  float* d = nullptr;  // device: theta | mean | scale | m | v | grad | sse
  int64_t t = 0;       // Adam steps taken
  float* theta() const { return d; }
  float* mean() const { return d + ffx::MLP_NPARAM; }
  float* scale() const { return d + ffx::MLP_NPARAM + ffx::MLP_NIN; }
  float* m() const { return d + ffx::MLP_NPARAM + 2 * ffx::MLP_NIN; }
  float* v() const { return m() + ffx::MLP_NPARAM; }
  float* grad() const { return v() + ffx::MLP_NPARAM; }
  float* sse() const { return grad() + ffx::MLP_NPARAM; }
  static size_t floats() { return 4 * ffx::MLP_NPARAM + 2 * ffx::MLP_NIN + 1; }
};

namespace ffx {

namespace {

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

ffx_selector_s* new_selector() {
  ffx_selector_s* S = new ffx_selector_s();
  if (hipMalloc(&S->d, ffx_selector_s::floats() * sizeof(float)) != hipSuccess) {
    delete S;
    fail(FFX_ENOMEM, "selector allocation failed");
  }
  if (hipMemset(S->d, 0, ffx_selector_s::floats() * sizeof(float)) != hipSuccess) {
    (void)hipFree(S->d);
    delete S;
    fail(FFX_EDEVICE, "selector initialisation failed");
  }
  return S;
}

// file: magic, count, mean[32], scale[32], theta[6662], FNV-1a of the float bytes
const char MAGIC[8] = {'F', 'F', 'X', 'M', 'L', 'P', '1', '\0'};
uint32_t fnv1a(const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  uint32_t h = 2166136261u;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 16777619u;
  return h;
}

bool read_model(const char* path, std::vector<float>& host) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  char magic[8];
  uint32_t count = 0, sum = 0;
  host.assign(MLP_NPARAM + 2 * MLP_NIN, 0.f);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, MAGIC, 8) == 0 && fread(&count, 4, 1, f) == 1 &&
            count == (uint32_t)host.size() && fread(host.data(), 4, host.size(), f) == host.size() &&
            fread(&sum, 4, 1, f) == 1 && sum == fnv1a(host.data(), host.size() * 4);
  fclose(f);
  if (ok)
    for (float v : host)
      if (!std::isfinite(v)) ok = false;
  return ok;
}

}  // namespace

// Build-time hook: predicted fastest format per block, or false (heuristic).
bool learned_formats(const std::string& model_path, const std::vector<BlockStats>& blocks, std::vector<int32_t>& fmt,
                     hipStream_t st) {
  if (model_path.empty() || blocks.empty()) return false;
  std::vector<float> host;  // mean | scale | theta as stored
  if (!read_model(model_path.c_str(), host)) return false;
  const int64_t n = (int64_t)blocks.size();
  std::vector<float> X(n * MLP_NIN);
  for (int64_t b = 0; b < n; ++b) memcpy(&X[b * MLP_NIN], blocks[b].feat, sizeof(float) * MLP_NIN);
  float* d = nullptr;
  size_t floats = host.size() + X.size() + n * MLP_NOUT;
  if (hipMalloc(&d, floats * sizeof(float)) != hipSuccess) return false;
  float* dmean = d;
  float* dscale = d + MLP_NIN;
  float* dtheta = d + 2 * MLP_NIN;
  float* dX = d + host.size();
  float* dout = dX + X.size();
  std::vector<float> out(n * MLP_NOUT);
  bool ok = hipMemcpyAsync(d, host.data(), host.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
            mlp_predict(dtheta, dmean, dscale, dX, n, dout, st) == hipSuccess &&
            hipMemcpyAsync(out.data(), dout, out.size() * 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
            hipStreamSynchronize(st) == hipSuccess;
  (void)hipFree(d);
  if (!ok) return false;
  for (int64_t b = 0; b < n; ++b) {
    int best = -1;
    float bv = INFINITY;
    for (int f = 0; f < MLP_NOUT; ++f) {
      float v = out[b * MLP_NOUT + f];
      if (!std::isfinite(v)) return false;  // a non-finite score: keep the heuristic
      if (v < bv) {
        bv = v;
        best = f;
      }
    }
    fmt[b] = best;
  }
  return true;
}

}  // namespace ffx

using namespace ffx;

extern "C" {

ffx_status ffx_selector_create(uint64_t seed, ffx_selector* out) {
  return guard([&] {
    if (!out) fail(FFX_EINVAL, "out is NULL");
    *out = nullptr;
    ffx_selector_s* S = new_selector();
    std::vector<float> theta(MLP_NPARAM, 0.f), scale(MLP_NIN, 1.f);
    // He-uniform weights: bound sqrt(6 / fan_in); biases 0
    const int fan[3][3] = {{0, 64 * 32, 32}, {64 * 32 + 64, 64 * 64, 64}, {64 * 32 + 64 + 64 * 64 + 64, 6 * 64, 64}};
    uint64_t ctr = 0;
    for (auto& w : fan) {
      float bound = std::sqrt(6.0f / (float)w[2]);
      for (int i = 0; i < w[1]; ++i) {
        double u = (double)(mix64(seed + (++ctr) * 0x9E3779B97F4A7C15ULL) >> 11) * (1.0 / 9007199254740992.0);
        theta[w[0] + i] = (float)((2.0 * u - 1.0) * bound);
      }
    }
    if (hipMemcpy(S->theta(), theta.data(), MLP_NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->scale(), scale.data(), MLP_NIN * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(S->d);
      delete S;
      fail(FFX_EDEVICE, "selector upload failed");
    }
    *out = S;
  });
}

ffx_status ffx_selector_set_params(ffx_selector S, const float* theta, const float* mean, const float* scale) {
  return guard([&] {
    if (!S) fail(FFX_EINVAL, "selector is NULL");
    if (theta) FFX_HIP(hipMemcpy(S->theta(), theta, MLP_NPARAM * 4, hipMemcpyHostToDevice));
    if (mean) FFX_HIP(hipMemcpy(S->mean(), mean, MLP_NIN * 4, hipMemcpyHostToDevice));
    if (scale) FFX_HIP(hipMemcpy(S->scale(), scale, MLP_NIN * 4, hipMemcpyHostToDevice));
  });
}

ffx_status ffx_selector_get_params(ffx_selector S, float* theta, float* mean, float* scale) {
  return guard([&] {
    if (!S) fail(FFX_EINVAL, "selector is NULL");
    if (theta) FFX_HIP(hipMemcpy(theta, S->theta(), MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    if (mean) FFX_HIP(hipMemcpy(mean, S->mean(), MLP_NIN * 4, hipMemcpyDeviceToHost));
    if (scale) FFX_HIP(hipMemcpy(scale, S->scale(), MLP_NIN * 4, hipMemcpyDeviceToHost));
  });
}

ffx_status ffx_selector_predict(ffx_selector S, const float* X, int64_t n, float* out, void* stream) {
  return guard([&] {
    if (!S || (n > 0 && (!X || !out)) || n < 0) fail(FFX_EINVAL, "bad argument");
    FFX_HIP(mlp_predict(S->theta(), S->mean(), S->scale(), X, n, out, (hipStream_t)stream));
  });
}

static void gradient(ffx_selector S, const float* X, const float* T, const float* M, int64_t n, float* grad,
                     double* loss, hipStream_t st) {
  if (!S || n < 1 || !X || !T || !M || !grad) fail(FFX_EINVAL, "bad argument");
  float* ws = nullptr;
  size_t floats = (size_t)n * (mlp_act_floats() + mlp_del_floats() + 1);
  if (hipMallocAsync((void**)&ws, floats * 4, st) != hipSuccess) fail(FFX_ENOMEM, "gradient workspace");
  float* act = ws;
  float* del = act + (size_t)n * mlp_act_floats();
  float* sq = del + (size_t)n * mlp_del_floats();
  hipError_t e = mlp_gradient(S->theta(), S->mean(), S->scale(), X, T, M, n, act, del, sq, grad, S->sse(), st);
  (void)hipFreeAsync(ws, st);
  FFX_HIP(e);
  if (loss) {
    float sse = 0;
    FFX_HIP(hipMemcpyAsync(&sse, S->sse(), 4, hipMemcpyDeviceToHost, st));
    FFX_HIP(hipStreamSynchronize(st));
    *loss = 0.5 * (double)sse / (double)n;
  }
}

ffx_status ffx_selector_gradient(ffx_selector S, const float* X, const float* T, const float* M, int64_t n,
                                 float* grad, double* loss, void* stream) {
  return guard([&] { gradient(S, X, T, M, n, grad, loss, (hipStream_t)stream); });
}

ffx_status ffx_selector_train_step(ffx_selector S, const float* X, const float* T, const float* M, int64_t n, float lr,
                                   double* loss, void* stream) {
  return guard([&] {
    hipStream_t st = (hipStream_t)stream;
    gradient(S, X, T, M, n, S ? S->grad() : nullptr, loss, st);
    S->t += 1;
    FFX_HIP(mlp_adam(S->theta(), S->m(), S->v(), S->grad(), lr, S->t, st));
  });
}

ffx_status ffx_selector_save(ffx_selector S, const char* path) {
  return guard([&] {
    if (!S || !path) fail(FFX_EINVAL, "bad argument");
    std::vector<float> host(MLP_NPARAM + 2 * MLP_NIN);
    FFX_HIP(hipMemcpy(host.data(), S->mean(), MLP_NIN * 4, hipMemcpyDeviceToHost));
    FFX_HIP(hipMemcpy(host.data() + MLP_NIN, S->scale(), MLP_NIN * 4, hipMemcpyDeviceToHost));
    FFX_HIP(hipMemcpy(host.data() + 2 * MLP_NIN, S->theta(), MLP_NPARAM * 4, hipMemcpyDeviceToHost));
    FILE* f = fopen(path, "wb");
    if (!f) fail(FFX_EINVAL, "cannot write %s", path);
    uint32_t count = (uint32_t)host.size(), sum = fnv1a(host.data(), host.size() * 4);
    bool ok = fwrite(MAGIC, 1, 8, f) == 8 && fwrite(&count, 4, 1, f) == 1 &&
              fwrite(host.data(), 4, host.size(), f) == host.size() && fwrite(&sum, 4, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) fail(FFX_EINVAL, "short write to %s", path);
  });
}

ffx_status ffx_selector_load(const char* path, ffx_selector* out) {
  return guard([&] {
    if (!path || !out) fail(FFX_EINVAL, "bad argument");
    *out = nullptr;
    std::vector<float> host;
    if (!read_model(path, host)) fail(FFX_EINVAL, "%s is not a valid selector model", path);
    ffx_selector_s* S = new_selector();
    if (hipMemcpy(S->mean(), host.data(), MLP_NIN * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->scale(), host.data() + MLP_NIN, MLP_NIN * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S->theta(), host.data() + 2 * MLP_NIN, MLP_NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(S->d);
      delete S;
      fail(FFX_EDEVICE, "selector upload failed");
    }
    *out = S;
  });
}

ffx_status ffx_selector_destroy(ffx_selector S) {
  return guard([&] {
    if (!S) return;
    (void)hipFree(S->d);
    delete S;
  });
}

}  // extern "C"
