// Autotuner for the sample-axis tiling of the batched kernels.
//
// For one call kind it times every supported (S, chunk length, ordering)
// candidate on the caller's own population with HIP events, applies the
// fastest, and can persist the choice in a plain-text cache, one line per
// (device architecture, model, T, kind, k_max):
//     <arch> <model> <T> <kind> <k_max> <S> <chunk_len> <sorted> <ms>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "smcx_problem.h"

namespace {

struct Candidate {
  int S;
  int64_t chunk;
  int sorted;
};

std::vector<Candidate> candidates(const smcx_problem* p, int kind) {
  std::vector<Candidate> out;
  const std::vector<int> Ss = kind == kDelta ? std::vector<int>{8, 16} : std::vector<int>{8, 16, 32, 64};
  for (int S : Ss) {
    const int64_t tile = 64 * (int64_t)S;
    std::vector<int64_t> chunks = {(p->T + tile - 1) / tile * tile};
    for (int64_t c : {2048, 4096, 8192, 16384, 32768, 65536})
      if (c % tile == 0 && c < p->T) chunks.push_back(c);
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
    for (int64_t c : chunks) {
      const int nch = (int)((p->T + c - 1) / c);
      if (nch > p->max_nch) continue;
      if (kind == kGrad && nch > 1 && nch > p->max_nch_grad) continue;
      // the persistent grid (2) serves the logL and gradient kernels
      for (int so : {0, 1, 2})
        if (so < 2 || kind != kDelta) out.push_back({S, c, so});
    }
  }
  return out;
}

std::string cache_key(const smcx_problem* p, int kind) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  std::ostringstream os;
  os << arch << " " << p->model << " " << p->T << " " << kind << " " << p->k_max;
  return os.str();
}

bool cache_lookup(const char* path, const std::string& key, Candidate& c, double& ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.compare(0, key.size() + 1, key + " ") != 0) continue;
    std::istringstream is(line.substr(key.size() + 1));
    Candidate t;
    double m;
    if (is >> t.S >> t.chunk >> t.sorted >> m) {
      c = t;
      ms = m;
      found = true;  // the last matching line wins
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const Candidate& c, double ms) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << c.S << " " << c.chunk << " " << c.sorted << " " << ms << "\n";
}

}  // namespace

extern "C" int smcx_autotune(smcx_problem* p, int32_t kind, int64_t N, const int64_t* offsets,
                             int64_t M, const double* theta, const double* beta, int32_t reps,
                             const char* cache_path, void* hip_stream, int32_t* out_S,
                             int64_t* out_chunk, int32_t* out_sorted, double* out_ms) {
  if (!p) return smcx::set_error(SMCX_EINVAL, "problem handle is NULL");
  if (p->fd) return smcx::set_error(SMCX_EINVAL, "frequency-domain problems have no sample tiling");
  if (kind < 0 || kind >= kNumKinds) return smcx::set_error(SMCX_EINVAL, "unknown call kind %d", kind);
  if (reps < 1 || reps > 1000) return smcx::set_error(SMCX_EINVAL, "reps out of range");
  if (N < 1 || N > p->n_max || M < 1 || M > p->m_max || !offsets || !theta)
    return smcx::set_error(SMCX_EINVAL, "autotune needs a population with N >= 1 and M >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return smcx::set_error(SMCX_ECAPTURE, "smcx_autotune called during stream capture");

  const std::string key = cache_key(p, kind);
  Candidate best{0, 0, 0};
  double best_ms = 0.0;
  if (cache_lookup(cache_path, key, best, best_ms) &&
      smcx_set_tiling(p, kind, best.S, best.chunk, best.sorted) == SMCX_OK) {
    if (out_S) *out_S = best.S;
    if (out_chunk) *out_chunk = best.chunk;
    if (out_sorted) *out_sorted = best.sorted;
    if (out_ms) *out_ms = best_ms;
    return SMCX_OK;
  }

  // scratch outputs (and a birth row per particle for the birth/death pass)
  const int P = p->P;
  double *o1 = nullptr, *o2 = nullptr, *tb = nullptr;
  hipError_t e = hipMalloc(&o1, (size_t)N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&o2, (size_t)std::max<int64_t>(M, N) * P * sizeof(double));
  if (e == hipSuccess && kind == kDelta) {
    e = hipMalloc(&tb, (size_t)N * P * sizeof(double));
    // birth candidates: the population's own component rows, repeated
    for (int64_t i = 0; e == hipSuccess && i < N; i += M) {
      const int64_t n = std::min<int64_t>(M, N - i);
      e = hipMemcpyAsync(tb + i * P, theta, n * P * sizeof(double), hipMemcpyDeviceToDevice, st);
    }
  }
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFree(o1);
    (void)hipFree(o2);
    (void)hipFree(tb);
  };
  if (e != hipSuccess) {
    cleanup();
    return smcx::set_error(SMCX_ENOMEM, "autotune scratch allocation failed: %s", hipGetErrorString(e));
  }
  auto call = [&]() -> int {
    switch (kind) {
      case kGrad: return logl_grad_batch(p, N, offsets, M, theta, beta, o1, o2, st);
      case kFwd: return logl_batch(p, N, offsets, M, theta, beta, o1, st);
      default: return delta_logl_birth_death(p, N, offsets, M, theta, beta, tb, nullptr, o1, nullptr, st);
    }
  };

  const Tiling saved = p->tiling[kind];
  best_ms = INFINITY;
  int rc = SMCX_OK;
  for (const Candidate& c : candidates(p, kind)) {
    if (smcx_set_tiling(p, kind, c.S, c.chunk, c.sorted) != SMCX_OK) continue;
    rc = call();  // warm-up
    if (rc != SMCX_OK) break;
    e = hipEventRecord(ev0, st);
    for (int r = 0; r < reps && rc == SMCX_OK && e == hipSuccess; ++r) rc = call();
    if (e == hipSuccess) e = hipEventRecord(ev1, st);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (rc != SMCX_OK || e != hipSuccess) break;
    const double per = ms / reps;
    if (per < best_ms) {
      best_ms = per;
      best = c;
    }
  }
  cleanup();
  if (rc != SMCX_OK || e != hipSuccess || !std::isfinite(best_ms)) {
    p->tiling[kind] = saved;
    if (rc == SMCX_OK)
      rc = smcx::set_error(SMCX_EDEVICE, "autotune timing failed: %s", hipGetErrorString(e));
    return rc;
  }
  rc = smcx_set_tiling(p, kind, best.S, best.chunk, best.sorted);
  if (rc != SMCX_OK) return rc;
  cache_store(cache_path, key, best, best_ms);
  if (out_S) *out_S = best.S;
  if (out_chunk) *out_chunk = best.chunk;
  if (out_sorted) *out_sorted = best.sorted;
  if (out_ms) *out_ms = best_ms;
  return SMCX_OK;
}
