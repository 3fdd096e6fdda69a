// Training of the learned format selector inside the library: labels measured
// on this GPU, then standardisation, minibatch Adam with a cosine-decayed rate
// on the library's MLP kernels, and the choice of a decision margin on held-out
// samples. The paper's chooser is a hand heuristic whose thresholds have to be
// tuned per machine (Section 2.4, "Heuristic format chooser"); this replaces
// the hand tuning by measurement.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"
#include "mlp.h"

namespace ffx {
namespace {

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void check(ffx_status st) {
  if (st != FFX_OK) fail(st, "%s", ffx_last_error());
}

// Device buffer freed on scope exit.
struct DevBuf {
  void* p = nullptr;
  explicit DevBuf(size_t bytes) {
    if (bytes && hipMalloc(&p, bytes) != hipSuccess) fail(FFX_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const { return (T*)p; }
};

struct MatrixGuard {
  ffx_matrix M = nullptr;
  ~MatrixGuard() {
    if (M) (void)ffx_matrix_destroy(M);
  }
};

struct SelectorGuard {
  ffx_selector S = nullptr;
  ~SelectorGuard() {
    if (S) (void)ffx_selector_destroy(S);
  }
};

// Median microseconds of the in-place product y = A x over reps launches on st.
double time_product(ffx_matrix M, const void* x, void* y, int reps, hipStream_t st) {
  for (int w = 0; w < 2; ++w) check(ffx_spmv(M, 1, x, 0, y, FFX_I32, st));
  hipEvent_t e0, e1;
  FFX_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    fail(FFX_EDEVICE, "hipEventCreate failed");
  }
  std::vector<double> us;
  hipError_t e = hipSuccess;
  ffx_status fs = FFX_OK;
  for (int r = 0; r < reps && e == hipSuccess && fs == FFX_OK; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) fs = ffx_spmv(M, 1, x, 0, y, FFX_I32, st);
    if (e == hipSuccess && fs == FFX_OK) e = hipEventRecord(e1, st);
    if (e == hipSuccess && fs == FFX_OK) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess && fs == FFX_OK) e = hipEventElapsedTime(&ms, e0, e1);
    us.push_back(ms * 1000.0);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  check(fs);
  FFX_HIP(e);
  std::sort(us.begin(), us.end());
  return us[us.size() / 2];
}

// Summed time of a per-sample choice relative to the best per sample (1 = best), from log2 labels.
double choice_cost(const float* T, const std::vector<int>& choice, int64_t n) {
  double got = 0, best = 0;
  for (int64_t i = 0; i < n; ++i) {
    const float* t = T + i * MLP_NOUT;
    got += std::exp2((double)t[choice[i]]);
    double b = INFINITY;
    for (int f = 0; f < MLP_NOUT; ++f) b = std::min(b, std::exp2((double)t[f]));
    best += b;
  }
  return best > 0 ? got / best : 1.0;
}

}  // namespace
}  // namespace ffx

using namespace ffx;

extern "C" {

void ffx_train_opts_default(ffx_train_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->size = sizeof *o;
  o->epochs = 60;
  o->batch = 512;
  o->lr = 2e-3f;
  o->seed = 0;
  o->n_val = -1;
  o->n_margins = 0;
  o->margins = nullptr;
}

ffx_status ffx_selector_label(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                              const void* vals, ffx_dtype val_type, uint32_t m, const ffx_build_opts* opts,
                              int32_t reps, uint64_t seed, void* stream, int64_t cap, float* feat, float* labels,
                              int32_t* heur, int64_t* nblocks) {
  return guard([&] {
    if (!feat || !labels) fail(FFX_EINVAL, "NULL output");
    if (reps < 1 || reps > 10000) fail(FFX_EINVAL, "reps = %d outside [1, 10000]", reps);
    if (m > 65536u) fail(FFX_EUNSUPPORTED, "labels are timed with int32 vectors of residues below 65536");
    hipStream_t st = (hipStream_t)stream;
    ffx_build_opts o;
    ffx_build_opts_default(&o);
    if (opts) {
      if (opts->size < sizeof(uint32_t) || opts->size > sizeof o) fail(FFX_EINVAL, "ffx_build_opts.size = %u", opts->size);
      std::memcpy(&o, opts, opts->size);
      o.size = sizeof o;
    }
    int64_t nb = 0;
    check(ffx_block_features(nrows, ncols, rowptr, colidx, vals, val_type, m, &o, nullptr, 0, &nb));
    if (nblocks) *nblocks = nb;
    if (cap < nb) fail(FFX_EINVAL, "outputs hold %lld blocks, the window has %lld", (long long)cap, (long long)nb);
    if (nb == 0) return;
    check(ffx_block_features(nrows, ncols, rowptr, colidx, vals, val_type, m, &o, feat, cap, nullptr));
    // x: residues drawn from the seed; y: the product's rows
    std::vector<int32_t> xh((size_t)std::max<int64_t>(ncols, 1));
    uint64_t s = seed;
    for (auto& v : xh) v = (int32_t)(splitmix(s) % m);
    DevBuf dx(xh.size() * 4), dy((size_t)std::max<int64_t>(nrows, 1) * 4);
    FFX_HIP(hipMemcpyAsync(dx.p, xh.data(), xh.size() * 4, hipMemcpyHostToDevice, st));
    o.col_sorted = 0;  // the labels time the block formats: one-vector products on the tiles
    for (int f = 0; f < FFX_NUM_FORMATS; ++f) {
      o.selector = FFX_SEL_FIXED;
      o.fixed_format = f;
      MatrixGuard g;
      check(ffx_matrix_create_csr(nrows, ncols, rowptr, colidx, vals, val_type, m, &o, st, &g.M));
      const double us = time_product(g.M, dx.p, dy.p, reps, st);
      const float lab = (float)std::log2(std::max(us / (double)nb, 1e-3));
      for (int64_t b = 0; b < nb; ++b) labels[b * FFX_NUM_FORMATS + f] = lab;
    }
    if (heur) {
      o.selector = FFX_SEL_HEURISTIC;
      MatrixGuard g;
      check(ffx_matrix_create_csr(nrows, ncols, rowptr, colidx, vals, val_type, m, &o, st, &g.M));
      check(ffx_matrix_block_formats(g.M, 0, heur, nb));
    }
  });
}

ffx_status ffx_selector_train(const float* X, const float* T, const float* mask, const int32_t* heur, int64_t n,
                              const ffx_train_opts* opts, const char* out_model, ffx_selector* out,
                              ffx_train_report* report, void* stream) {
  return guard([&] {
    if (out) *out = nullptr;
    if (!X || !T) fail(FFX_EINVAL, "NULL samples");
    ffx_train_opts o;
    ffx_train_opts_default(&o);
    if (opts) {
      if (opts->size < sizeof(uint32_t) || opts->size > sizeof o) fail(FFX_EINVAL, "ffx_train_opts.size = %u", opts->size);
      std::memcpy(&o, opts, opts->size);
      o.size = sizeof o;
    }
    const int64_t nval = o.n_val < 0 ? n / 10 : o.n_val;
    const int64_t ntr = n - nval;
    if (nval < 1 || ntr < 2) fail(FFX_EINVAL, "%lld samples with %lld held out: need >= 1 held out and >= 2 to train",
                                  (long long)n, (long long)nval);
    if (o.epochs < 1 || o.epochs > 100000) fail(FFX_EINVAL, "epochs = %d", o.epochs);
    if (o.batch < 2) fail(FFX_EINVAL, "batch = %d < 2", o.batch);
    if (!(o.lr > 0) || !std::isfinite(o.lr)) fail(FFX_EINVAL, "learning rate %g", (double)o.lr);
    static const float default_margins[] = {0.f, 0.05f, 0.1f, 0.2f, 0.3f, 0.5f};
    const float* margins = o.n_margins > 0 ? o.margins : default_margins;
    const int nm = o.n_margins > 0 ? o.n_margins : 6;
    if (o.n_margins > 0 && !o.margins) fail(FFX_EINVAL, "margins is NULL");
    for (int k = 0; k < nm; ++k)
      if (!std::isfinite(margins[k])) fail(FFX_EINVAL, "margin %d is not finite", k);
    for (int64_t i = 0; i < n * MLP_NIN; ++i)
      if (!std::isfinite(X[i])) fail(FFX_EINVAL, "feature %lld is not finite", (long long)i);
    for (int64_t i = 0; i < n * MLP_NOUT; ++i)
      if (!std::isfinite(T[i])) fail(FFX_EINVAL, "label %lld is not finite", (long long)i);
    hipStream_t st = (hipStream_t)stream;

    // standardisation from the training samples: x' = (x - mean) * scale
    std::vector<float> mean(MLP_NIN), scale(MLP_NIN);
    for (int j = 0; j < MLP_NIN; ++j) {
      double s1 = 0, s2 = 0;
      for (int64_t i = nval; i < n; ++i) {
        double v = X[i * MLP_NIN + j];
        s1 += v;
        s2 += v * v;
      }
      const double mu = s1 / (double)ntr, sd = std::sqrt(std::max(0.0, s2 / (double)ntr - mu * mu));
      mean[j] = (float)mu;
      scale[j] = sd > 1e-6 ? (float)(1.0 / sd) : 1.f;
    }
    // targets relative to STREAM (output 0): the choice only depends on differences between formats
    std::vector<float> R((size_t)n * MLP_NOUT), Mk((size_t)n * MLP_NOUT, 1.f);
    for (int64_t i = 0; i < n; ++i)
      for (int f = 0; f < MLP_NOUT; ++f) {
        R[i * MLP_NOUT + f] = T[i * MLP_NOUT + f] - T[i * MLP_NOUT];
        if (mask) Mk[i * MLP_NOUT + f] = mask[i * MLP_NOUT + f] != 0.f ? 1.f : 0.f;
      }

    SelectorGuard sg;
    check(ffx_selector_create(o.seed, &sg.S));
    check(ffx_selector_set_params(sg.S, nullptr, mean.data(), scale.data()));
    const size_t rowb = (size_t)(MLP_NIN + 2 * MLP_NOUT) * 4;
    DevBuf dtr((size_t)ntr * rowb), dval((size_t)nval * rowb), dpred((size_t)nval * MLP_NOUT * 4);
    float* tX = dtr.as<float>();
    float* tT = tX + ntr * MLP_NIN;
    float* tM = tT + ntr * MLP_NOUT;
    float* vX = dval.as<float>();
    float* vT = vX + nval * MLP_NIN;
    float* vM = vT + nval * MLP_NOUT;
    FFX_HIP(hipMemcpyAsync(vX, X, nval * MLP_NIN * 4, hipMemcpyHostToDevice, st));
    FFX_HIP(hipMemcpyAsync(vT, R.data(), nval * MLP_NOUT * 4, hipMemcpyHostToDevice, st));
    FFX_HIP(hipMemcpyAsync(vM, Mk.data(), nval * MLP_NOUT * 4, hipMemcpyHostToDevice, st));

    // minibatch Adam, samples reshuffled every epoch, rate lr * (1 + cos(pi * epoch / epochs)) / 2
    std::vector<int64_t> perm(ntr);
    for (int64_t i = 0; i < ntr; ++i) perm[i] = nval + i;
    std::vector<float> hX((size_t)ntr * MLP_NIN), hT((size_t)ntr * MLP_NOUT), hM((size_t)ntr * MLP_NOUT);
    uint64_t rs = o.seed ^ 0x5EEDF00DULL;
    int32_t steps = 0;
    for (int ep = 0; ep < o.epochs; ++ep) {
      for (int64_t i = ntr - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(splitmix(rs) % (uint64_t)(i + 1))]);
      for (int64_t i = 0; i < ntr; ++i) {
        std::memcpy(&hX[i * MLP_NIN], X + perm[i] * MLP_NIN, MLP_NIN * 4);
        std::memcpy(&hT[i * MLP_NOUT], &R[perm[i] * MLP_NOUT], MLP_NOUT * 4);
        std::memcpy(&hM[i * MLP_NOUT], &Mk[perm[i] * MLP_NOUT], MLP_NOUT * 4);
      }
      FFX_HIP(hipMemcpyAsync(tX, hX.data(), hX.size() * 4, hipMemcpyHostToDevice, st));
      FFX_HIP(hipMemcpyAsync(tT, hT.data(), hT.size() * 4, hipMemcpyHostToDevice, st));
      FFX_HIP(hipMemcpyAsync(tM, hM.data(), hM.size() * 4, hipMemcpyHostToDevice, st));
      const float lr = (float)(o.lr * 0.5 * (1.0 + std::cos(M_PI * (double)ep / (double)o.epochs)));
      for (int64_t b0 = 0; b0 < ntr; b0 += o.batch) {
        const int64_t cnt = std::min<int64_t>(o.batch, ntr - b0);
        if (cnt < 2) continue;
        check(ffx_selector_train_step(sg.S, tX + b0 * MLP_NIN, tT + b0 * MLP_NOUT, tM + b0 * MLP_NOUT, cnt, lr,
                                      nullptr, st));
        ++steps;
      }
      // the host copies are reused next epoch: the uploads must be done
      FFX_HIP(hipStreamSynchronize(st));
    }
    double train_loss = 0, val_loss = 0;
    {
      DevBuf g(MLP_NPARAM * 4);
      check(ffx_selector_gradient(sg.S, tX, tT, tM, ntr, g.as<float>(), &train_loss, st));
      check(ffx_selector_gradient(sg.S, vX, vT, vM, nval, g.as<float>(), &val_loss, st));
    }

    // decision margin: outputs 1..5 predicted mu slower, so a block leaves STREAM only for a
    // predicted gain above mu; the margin with the least held-out time is folded into the biases
    std::vector<float> P((size_t)nval * MLP_NOUT);
    check(ffx_selector_predict(sg.S, vX, nval, dpred.as<float>(), st));
    FFX_HIP(hipMemcpyAsync(P.data(), dpred.p, P.size() * 4, hipMemcpyDeviceToHost, st));
    FFX_HIP(hipStreamSynchronize(st));
    auto choose = [&](float mu) {
      std::vector<int> c(nval);
      for (int64_t i = 0; i < nval; ++i) {
        int best = 0;
        float bv = P[i * MLP_NOUT];
        for (int f = 1; f < MLP_NOUT; ++f) {
          float v = P[i * MLP_NOUT + f] + mu;
          if (v < bv) {
            bv = v;
            best = f;
          }
        }
        c[i] = best;
      }
      return c;
    };
    float best_mu = margins[0];
    double best_cost = INFINITY;
    for (int k = 0; k < nm; ++k) {
      double c = choice_cost(T, choose(margins[k]), nval);
      // ties (to 1e-4) go to the smaller margin
      if (c < best_cost - 1e-4 || (std::fabs(c - best_cost) <= 1e-4 && margins[k] < best_mu)) {
        best_cost = std::min(best_cost, c);
        best_mu = margins[k];
      }
    }
    std::vector<float> theta(MLP_NPARAM);
    check(ffx_selector_get_params(sg.S, theta.data(), nullptr, nullptr));
    for (int f = 1; f < MLP_NOUT; ++f) theta[MLP_NPARAM - MLP_NOUT + f] += best_mu;  // b3[1..5]
    check(ffx_selector_set_params(sg.S, theta.data(), nullptr, nullptr));
    if (report) {
      std::memset(report, 0, sizeof *report);
      report->train_loss = train_loss;
      report->val_loss = val_loss;
      report->margin = best_mu;
      report->val_cost = choice_cost(T, choose(best_mu), nval);
      report->val_cost_stream = choice_cost(T, std::vector<int>(nval, 0), nval);
      if (heur) {
        std::vector<int> h(nval);
        for (int64_t i = 0; i < nval; ++i) {
          if (heur[i] < 0 || heur[i] >= MLP_NOUT) fail(FFX_EINVAL, "heuristic format %d at %lld", heur[i], (long long)i);
          h[i] = heur[i];
        }
        report->val_cost_heuristic = choice_cost(T, h, nval);
      }
      report->steps = steps;
    }
    if (out_model) check(ffx_selector_save(sg.S, out_model));
    if (out) {
      *out = sg.S;
      sg.S = nullptr;
    }
  });
}

}  // extern "C"

extern "C" ffx_status ffx_tune_tile_entries(int64_t nrows, int64_t ncols, const int64_t* rowptr, const int32_t* colidx,
                                            const void* vals, ffx_dtype val_type, uint32_t m,
                                            const ffx_build_opts* opts, int32_t s, int32_t reps, uint64_t seed,
                                            void* stream, int32_t* best_tile_entries, float* us_out) {
  return guard([&] {
    if (!best_tile_entries) fail(FFX_EINVAL, "best_tile_entries is NULL");
    if (s < 1 || s > MAX_S) fail(FFX_EINVAL, "s = %d outside [1, %d]", s, MAX_S);
    if (reps < 1 || reps > 10000) fail(FFX_EINVAL, "reps = %d outside [1, 10000]", reps);
    if (m < 2 || m > 2147483647u) fail(FFX_EINVAL, "modulus %u", m);
    hipStream_t st = (hipStream_t)stream;
    ffx_build_opts o;
    ffx_build_opts_default(&o);
    if (opts) {
      if (opts->size < sizeof(uint32_t) || opts->size > sizeof o) fail(FFX_EINVAL, "ffx_build_opts.size = %u", opts->size);
      std::memcpy(&o, opts, opts->size);
      o.size = sizeof o;
    }
    o.col_sorted = 0;  // the tiles are what is tuned
    // X: ncols x s random residues (int32), Y: nrows x s
    std::vector<int32_t> xh((size_t)std::max<int64_t>(ncols, 1) * s);
    uint64_t r = seed;
    for (auto& v : xh) v = (int32_t)(splitmix(r) % m);
    DevBuf dx(xh.size() * 4), dy((size_t)std::max<int64_t>(nrows, 1) * s * 4);
    FFX_HIP(hipMemcpyAsync(dx.p, xh.data(), xh.size() * 4, hipMemcpyHostToDevice, st));
    static const int32_t cand[4] = {512, 1024, 2048, 4096};
    double best = INFINITY;
    int32_t pick = cand[2];
    for (int c = 0; c < 4; ++c) {
      o.tile_entries = cand[c];
      MatrixGuard g;
      check(ffx_matrix_create_csr(nrows, ncols, rowptr, colidx, vals, val_type, m, &o, st, &g.M));
      auto run = [&]() {
        return s == 1 ? ffx_spmv(g.M, 1, dx.p, 0, dy.p, FFX_I32, st)
                      : ffx_spmm(g.M, s, 1, dx.p, s, 0, dy.p, s, FFX_I32, st);
      };
      for (int w = 0; w < 2; ++w) check(run());
      hipEvent_t e0, e1;
      FFX_HIP(hipEventCreate(&e0));
      if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        fail(FFX_EDEVICE, "hipEventCreate failed");
      }
      std::vector<double> us;
      hipError_t e = hipSuccess;
      ffx_status fs = FFX_OK;
      for (int k = 0; k < reps && e == hipSuccess && fs == FFX_OK; ++k) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) fs = run();
        if (e == hipSuccess && fs == FFX_OK) e = hipEventRecord(e1, st);
        if (e == hipSuccess && fs == FFX_OK) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess && fs == FFX_OK) e = hipEventElapsedTime(&ms, e0, e1);
        us.push_back(ms * 1000.0);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      check(fs);
      FFX_HIP(e);
      std::sort(us.begin(), us.end());
      const double med = us[us.size() / 2];
      if (us_out) us_out[c] = (float)med;
      if (med < best) {
        best = med;
        pick = cand[c];
      }
    }
    *best_tile_entries = pick;
  });
}
