// tgks_batch.hip -- batched runs of many independent grids (include/tgks.h).
//
// One launch per kernel kind and stage covers every instance: the face and
// cell kernels walk (instance, local block) work lists, the CFL reduction
// ends with one block per instance.  A run of n steps can be captured into a
// HIP graph and replayed; the 2-D tile shape is chosen by timing every shape
// on the batch.
#include "tgks_batch.hpp"
#include "tgks_internal.hpp"

using namespace tgks;

struct tgks_batch {
  int D = 0, nc = 0, ninst = 0;
  bool ns = false;
  bool chr = false;  // characteristic reconstruction variables
  bool fb = false;   // first-order fallback
  int tile2 = 0;
  hipStream_t stream = nullptr;
  std::vector<BatchInst> host;   // per instance (offsets in doubles)
  std::vector<int64_t> woff;     // ninst + 1 state offsets
  long long total = 0;           // doubles of one packed state
  long long nface[2] = {0, 0};   // doubles of the face arrays per direction
  int ncblk = 0;                 // cell blocks
  BatchInst* inst = nullptr;
  int2* wcell = nullptr;         // cell work list
  int2* wface[NTILE2][2] = {};   // 2-D face work lists per tile shape and direction
  int nwface[NTILE2][2] = {};
  int2* wface1 = nullptr;        // 1-D face work list
  int nwface1 = 0;
  double *Ws = nullptr, *P = nullptr, *W2 = nullptr;
  double* FA[2] = {nullptr, nullptr};
  double* FB[2] = {nullptr, nullptr};
  double* partial = nullptr;
  double* clock = nullptr;
  long long* steps = nullptr;
  unsigned long long* fail = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int g_steps = -1;
  double g_cfl = 0, g_tend = 0;
  double* g_W = nullptr;
  double* g_time = nullptr;
};

static void drop_graph(tgks_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_steps = -1;
}

static void free_batch(tgks_batch* b) {
  if (!b) return;
  drop_graph(b);
  (void)hipFree(b->inst);
  (void)hipFree(b->wcell);
  for (int t = 0; t < NTILE2; ++t)
    for (int d = 0; d < 2; ++d) (void)hipFree(b->wface[t][d]);
  (void)hipFree(b->wface1);
  (void)hipFree(b->Ws);
  (void)hipFree(b->P);
  (void)hipFree(b->W2);
  for (int d = 0; d < 2; ++d) {
    (void)hipFree(b->FA[d]);
    (void)hipFree(b->FB[d]);
  }
  (void)hipFree(b->partial);
  (void)hipFree(b->clock);
  (void)hipFree(b->steps);
  (void)hipFree(b->fail);
  delete b;
}

template <class T>
static bool upload(T** dst, const std::vector<T>& v) {
  if (v.empty()) return true;
  if (hipMalloc(dst, v.size() * sizeof(T)) != hipSuccess) return false;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

static BatchArgs batch_args(tgks_batch* b, const double* W, double* o1, double* o2, const int2* work) {
  BatchArgs a;
  a.inst = b->inst;
  a.work = work;
  a.W = W;
  a.out1 = o1;
  a.out2 = o2;
  for (int d = 0; d < 2; ++d) {
    a.FA[d] = b->FA[d];
    a.FB[d] = b->FB[d];
  }
  a.clock = b->clock;
  a.partial = b->partial;
  a.fail = b->fail;
  a.fallback = b->fb ? 1 : 0;
  return a;
}

#define BLAUNCH(kern, nblk, threads, args) hipLaunchKernelGGL(kern, dim3((unsigned)(nblk)), dim3(threads), 0, b->stream, args)

template <int TILE, bool CHAR = false, bool EX = false>
static void batch_face2d(tgks_batch* b, const double* W, int ax, int stage) {
  constexpr int NT = 2 * tile2_tn(TILE) * tile2_tt(TILE);
  const int nw = b->nwface[TILE][ax];
  if (nw == 0) return;
  BatchArgs a = batch_args(b, W, nullptr, nullptr, b->wface[TILE][ax]);
#define BF2(AXV)                                                                                  \
  if (stage == 1) {                                                                               \
    if (b->ns) BLAUNCH((batch_face2d_kernel<AXV, 1, true, TILE, CHAR, EX>), nw, NT, a);               \
    else BLAUNCH((batch_face2d_kernel<AXV, 1, false, TILE, CHAR, EX>), nw, NT, a);                    \
  } else {                                                                                        \
    if (b->ns) BLAUNCH((batch_face2d_kernel<AXV, 2, true, TILE, CHAR, EX>), nw, NT, a);               \
    else BLAUNCH((batch_face2d_kernel<AXV, 2, false, TILE, CHAR, EX>), nw, NT, a);                    \
  }
  if (ax == 0) {
    BF2(0)
  } else {
    BF2(1)
  }
#undef BF2
}

static int batch_faces(tgks_batch* b, const double* W, int stage) {
  if (b->D == 1) {
    BatchArgs a = batch_args(b, W, nullptr, nullptr, b->wface1);
#define BF1(CH, EX)                                                                     \
  if (stage == 1) {                                                                     \
    if (b->ns) BLAUNCH((batch_face1d_kernel<1, true, CH, EX>), b->nwface1, 256, a);     \
    else BLAUNCH((batch_face1d_kernel<1, false, CH, EX>), b->nwface1, 256, a);          \
  } else {                                                                              \
    if (b->ns) BLAUNCH((batch_face1d_kernel<2, true, CH, EX>), b->nwface1, 256, a);     \
    else BLAUNCH((batch_face1d_kernel<2, false, CH, EX>), b->nwface1, 256, a);          \
  }
    if (b->chr && b->fb) {
      BF1(true, true)
    } else if (b->chr) {
      BF1(true, false)
    } else if (b->fb) {
      BF1(false, true)
    } else {
      BF1(false, false)
    }
#undef BF1
  } else {
    for (int ax = 0; ax < 2; ++ax) {
      if (b->chr || b->fb) {  // one tile shape on the characteristic / fallback path
        if (b->chr && b->fb) batch_face2d<CHAR_TILE2, true, true>(b, W, ax, stage);
        else if (b->chr) batch_face2d<CHAR_TILE2, true>(b, W, ax, stage);
        else batch_face2d<CHAR_TILE2, false, true>(b, W, ax, stage);
        continue;
      }
      switch (b->tile2) {
        case 1:
          batch_face2d<1>(b, W, ax, stage);
          break;
        case 2:
          batch_face2d<2>(b, W, ax, stage);
          break;
        default:
          batch_face2d<0>(b, W, ax, stage);
      }
    }
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static int batch_update(tgks_batch* b, int stage, const double* W, double* o1, double* o2) {
  BatchArgs a = batch_args(b, W, o1, o2, b->wcell);
  if (b->D == 1) {
    if (stage == 1) BLAUNCH((batch_update_kernel<1, 1, false>), b->ncblk, 256, a);
    else BLAUNCH((batch_update_kernel<1, 2, true>), b->ncblk, 256, a);
  } else {
    if (stage == 1) BLAUNCH((batch_update_kernel<2, 1, false>), b->ncblk, 256, a);
    else BLAUNCH((batch_update_kernel<2, 2, true>), b->ncblk, 256, a);
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static int batch_finalize(tgks_batch* b, double cfl, double t_end, int mode) {
  hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)b->ninst), dim3(256), 0, b->stream, b->inst, b->partial,
                     cfl, t_end, b->clock, b->steps, mode);
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static int batch_cfl_start(tgks_batch* b, const double* W, double cfl, double t_end) {
  BatchArgs a = batch_args(b, W, nullptr, nullptr, b->wcell);
  if (b->D == 1)
    BLAUNCH((batch_cfl_partial_kernel<1>), b->ncblk, 256, a);
  else
    BLAUNCH((batch_cfl_partial_kernel<2>), b->ncblk, 256, a);
  HIPCHK(hipGetLastError());
  return batch_finalize(b, cfl, t_end, 0);
}

static int batch_step(tgks_batch* b, const double* W, double* out) {
  int r;
  if ((r = batch_faces(b, W, 1))) return r;
  if ((r = batch_update(b, 1, W, b->Ws, b->P))) return r;
  if ((r = batch_faces(b, b->Ws, 2))) return r;
  return batch_update(b, 2, b->P, out, nullptr);
}

static int enqueue_batch_run(tgks_batch* b, double* W, int n_steps, double cfl, double t_end, double* time_dev) {
  int r;
  if ((r = batch_cfl_start(b, W, cfl, t_end))) return r;
  double* src = W;
  double* dst = b->W2;
  for (int s = 0; s < n_steps; ++s) {
    if ((r = batch_step(b, src, dst))) return r;
    if ((r = batch_finalize(b, cfl, t_end, 1))) return r;
    double* t = src;
    src = dst;
    dst = t;
  }
  if (src != W) HIPCHK(hipMemcpyAsync(W, src, (size_t)b->total * sizeof(double), hipMemcpyDeviceToDevice, b->stream));
  if (time_dev)
    HIPCHK(hipMemcpyAsync(time_dev, b->clock, 2 * (size_t)b->ninst * sizeof(double), hipMemcpyDeviceToDevice,
                          b->stream));
  return TGKS_OK;
}

extern "C" {

int tgks_batch_create(const tgks_params* p, int32_t n_inst, void* stream, tgks_batch** out) {
  if (!out || !p || n_inst < 1) return TGKS_EINVAL;
  *out = nullptr;
  const int D = p[0].ndim;
  if (D != 1 && D != 2) return TGKS_EINVAL;
  const bool ns = p[0].mu > 0.0 && p[0].prandtl != 1.0;
  for (int i = 0; i < n_inst; ++i) {
    if (check_params(&p[i]) || p[i].ndim != D || p[i].recon != p[0].recon) return TGKS_EINVAL;
    if (p[i].scheme != TGKS_SCHEME_TENO_D) return TGKS_EINVAL;  // TENO-D batches only
    if (has_prescribed(&p[i]) || p[i].fallback != p[0].fallback) return TGKS_EINVAL;
    if ((p[i].mu > 0.0 && p[i].prandtl != 1.0) != ns) return TGKS_EINVAL;
  }
  tgks_batch* b = new (std::nothrow) tgks_batch();
  if (!b) return TGKS_EHIP;
  b->D = D;
  b->nc = D + 2;
  b->ninst = n_inst;
  b->ns = ns;
  b->chr = p[0].recon == TGKS_RECON_CHARACTERISTIC;
  b->fb = p[0].fallback != 0;
  b->stream = (hipStream_t)stream;
  std::vector<int2> wcell, wface1, wface[NTILE2][2];
  long long woff = 0, foff[2] = {0, 0};
  int blk = 0;
  b->woff.push_back(0);
  for (int i = 0; i < n_inst; ++i) {
    BatchInst I;
    memset(&I, 0, sizeof(I));
    Geom& g = I.g;
    g.D = D;
    g.ncell = 1;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = d < D ? p[i].n[d] : 1;
      g.dx[d] = d < D ? p[i].dx[d] : 1.0;
      g.bclo[d] = p[i].bc_lo[d];
      g.bchi[d] = p[i].bc_hi[d];
      g.ncell *= g.n[d];
    }
    const double N = 2.0 / (p[i].gamma - 1.0);
    I.fc.N = N;
    I.fc.K = N - D;
    I.fc.mu = p[i].mu;
    I.fc.pr_fix = ns ? 1.0 / p[i].prandtl - 1.0 : 0.0;
    I.fc.c1 = p[i].c1;
    I.fc.c2 = p[i].c2;
    I.fc.tau_mode = p[i].tau_mode;
    I.tn = teno_cfg(p[i].ct1, p[i].ct2, p[i].eps, p[i].q);
    I.tt = teno_cfg(p[i].ct1_tan, p[i].ct2_tan, p[i].eps, p[i].q);
    I.gamma = p[i].gamma;
    I.mu = p[i].mu;
    I.woff = woff;
    woff += (long long)b->nc * g.ncell;
    b->woff.push_back(woff);
    for (int d = 0; d < D; ++d) {
      I.foff[d] = foff[d];
      long long nf = 1;
      for (int e = 0; e < D; ++e) nf *= (long long)(g.n[e] + (e == d));
      foff[d] += (long long)b->nc * nf;
    }
    const int nblk = (int)((g.ncell + 255) / 256);
    I.blk0 = blk;
    I.nblk = nblk;
    blk += nblk;
    for (int k = 0; k < nblk; ++k) wcell.push_back(make_int2(i, k));
    if (D == 1) {
      const int nb = (g.n[0] + 1 + 255) / 256;
      for (int k = 0; k < nb; ++k) wface1.push_back(make_int2(i, k));
    } else {
      for (int ax = 0; ax < 2; ++ax) {
        // one work list per tile shape; ntile is set with the shape
        for (int t = 0; t < NTILE2; ++t) {
          const int tn = tile2_tn(t), tt = tile2_tt(t);
          const int a = (g.n[ax] + 1 + tn - 1) / tn, c = (g.n[1 - ax] + tt - 1) / tt;
          for (int k = 0; k < a * c; ++k) wface[t][ax].push_back(make_int2(i, k));
        }
      }
    }
    b->host.push_back(I);
  }
  b->total = woff;
  b->nface[0] = foff[0];
  b->nface[1] = foff[1];
  b->ncblk = blk;
  b->nwface1 = (int)wface1.size();
  for (int t = 0; t < NTILE2; ++t)
    for (int d = 0; d < 2; ++d) b->nwface[t][d] = (int)wface[t][d].size();
  const size_t state = (size_t)b->total * sizeof(double);
  bool ok = hipMalloc(&b->Ws, state) == hipSuccess && hipMalloc(&b->P, state) == hipSuccess &&
            hipMalloc(&b->W2, state) == hipSuccess;
  for (int d = 0; d < D && ok; ++d)
    ok = hipMalloc(&b->FA[d], (size_t)b->nface[d] * sizeof(double)) == hipSuccess &&
         hipMalloc(&b->FB[d], (size_t)b->nface[d] * sizeof(double)) == hipSuccess;
  if (ok)
    ok = hipMalloc(&b->partial, (size_t)b->ncblk * sizeof(double)) == hipSuccess &&
         hipMalloc(&b->clock, 2 * (size_t)n_inst * sizeof(double)) == hipSuccess &&
         hipMalloc(&b->steps, (size_t)n_inst * sizeof(long long)) == hipSuccess &&
         hipMalloc(&b->fail, (size_t)n_inst * sizeof(unsigned long long)) == hipSuccess;
  if (ok) ok = upload(&b->wcell, wcell) && upload(&b->wface1, wface1);
  for (int t = 0; t < NTILE2 && ok; ++t)
    for (int d = 0; d < 2 && ok; ++d) ok = upload(&b->wface[t][d], wface[t][d]);
  if (ok) ok = hipMalloc(&b->inst, (size_t)n_inst * sizeof(BatchInst)) == hipSuccess;
  if (ok) {
    b->tile2 = -1;
    ok = tgks_batch_set_tile(b, 0) == TGKS_OK;
  }
  if (ok) {
    hipLaunchKernelGGL(zero_counters_kernel, dim3((unsigned)((n_inst + 255) / 256)), dim3(256), 0, b->stream, b->fail,
                       n_inst);
    ok = hipGetLastError() == hipSuccess;
  }
  if (ok) ok = hipStreamSynchronize(b->stream) == hipSuccess;
  if (!ok) {
    free_batch(b);
    return TGKS_EHIP;
  }
  *out = b;
  return TGKS_OK;
}

int tgks_batch_destroy(tgks_batch* b) {
  if (!b) return TGKS_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  free_batch(b);
  return TGKS_OK;
}

int tgks_batch_set_stream(tgks_batch* b, void* stream) {
  if (!b) return TGKS_EINVAL;
  b->stream = (hipStream_t)stream;
  drop_graph(b);
  return TGKS_OK;
}

int64_t tgks_batch_state_size(const tgks_batch* b) { return b ? (int64_t)b->total : TGKS_EINVAL; }

int tgks_batch_offsets(const tgks_batch* b, int64_t* offsets) {
  if (!b || !offsets) return TGKS_EINVAL;
  for (int i = 0; i <= b->ninst; ++i) offsets[i] = b->woff[i];
  return TGKS_OK;
}

int tgks_batch_set_tile(tgks_batch* b, int32_t tile) {
  if (!b || tile < -1 || tile >= NTILE2) return TGKS_EINVAL;
  const int t = (b->chr || b->fb) ? CHAR_TILE2 : (tile < 0 ? 0 : tile);  // one shape: characteristic / fallback
  if (t == b->tile2) return TGKS_OK;
  drop_graph(b);
  // tiles along the normal axis of each direction for this shape
  for (auto& I : b->host)
    for (int ax = 0; ax < 2; ++ax) I.ntile[ax] = (I.g.n[ax] + 1 + tile2_tn(t) - 1) / tile2_tn(t);
  HIPCHK(hipStreamSynchronize(b->stream));
  HIPCHK(hipMemcpy(b->inst, b->host.data(), b->host.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
  b->tile2 = t;
  return TGKS_OK;
}

int tgks_batch_run(tgks_batch* b, double* W, int32_t n_steps, double cfl, double t_end, double* time_dev,
                   int32_t use_graph) {
  if (!b || !W || n_steps < 0 || !(cfl > 0.0)) return TGKS_EINVAL;
  if (!use_graph || b->stream == nullptr) return enqueue_batch_run(b, W, n_steps, cfl, t_end, time_dev);
  const bool same = b->gexec && b->g_steps == n_steps && b->g_cfl == cfl && b->g_tend == t_end && b->g_W == W &&
                    b->g_time == time_dev;
  if (!same) {
    drop_graph(b);
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int r = enqueue_batch_run(b, W, n_steps, cfl, t_end, time_dev);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (r) {
      if (gr) (void)hipGraphDestroy(gr);
      return r;
    }
    if (e != hipSuccess) {
      fprintf(stderr, "tgks: graph capture failed: %s\n", hipGetErrorString(e));
      return TGKS_EHIP;
    }
    b->graph = gr;
    HIPCHK(hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0));
    b->g_steps = n_steps;
    b->g_cfl = cfl;
    b->g_tend = t_end;
    b->g_W = W;
    b->g_time = time_dev;
  }
  HIPCHK(hipGraphLaunch(b->gexec, b->stream));
  return TGKS_OK;
}

int tgks_batch_status(tgks_batch* b, int64_t* failures) {
  if (!b || !failures) return TGKS_EINVAL;
  std::vector<unsigned long long> h(b->ninst);
  HIPCHK(hipMemcpyAsync(h.data(), b->fail, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->ninst; ++i) failures[i] = (int64_t)h[i];
  return TGKS_OK;
}

int tgks_batch_steps(tgks_batch* b, int64_t* steps) {
  if (!b || !steps) return TGKS_EINVAL;
  std::vector<long long> h(b->ninst);
  HIPCHK(hipMemcpyAsync(h.data(), b->steps, h.size() * sizeof(long long), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->ninst; ++i) steps[i] = (int64_t)h[i];
  return TGKS_OK;
}

int tgks_batch_reset_status(tgks_batch* b) {
  if (!b) return TGKS_EINVAL;
  hipLaunchKernelGGL(zero_counters_kernel, dim3((unsigned)((b->ninst + 255) / 256)), dim3(256), 0, b->stream, b->fail,
                     b->ninst);
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

int tgks_batch_tune(tgks_batch* b, const double* W, int32_t steps, int32_t* chosen, float* ms_per_variant) {
  if (!b || !W || steps < 1) return TGKS_EINVAL;
  const int nvar = b->D == 2 ? NTILE2 : 1;
  int r;
  if ((r = batch_cfl_start(b, W, 0.5, 0.0))) return r;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const int old = b->tile2;
  int best = (b->chr || b->fb) ? CHAR_TILE2 : 0;
  float best_ms = 0.f;
  bool first = true;
  for (int k = 0; k < nvar && !r; ++k) {
    if ((b->chr || b->fb) && k != CHAR_TILE2) {  // one tile shape on the characteristic / fallback path
      if (ms_per_variant) ms_per_variant[k] = 0.f;
      continue;
    }
    if ((r = tgks_batch_set_tile(b, k))) break;
    if ((r = batch_step(b, W, b->W2))) break;  // warm-up
    if (hipEventRecord(e0, b->stream) != hipSuccess) r = TGKS_EHIP;
    for (int s = 0; s < steps && !r; ++s) r = batch_step(b, W, b->W2);
    if (!r && hipEventRecord(e1, b->stream) != hipSuccess) r = TGKS_EHIP;
    if (!r && hipEventSynchronize(e1) != hipSuccess) r = TGKS_EHIP;
    float ms = 0.f;
    if (!r && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) r = TGKS_EHIP;
    if (r) break;
    if (ms_per_variant) ms_per_variant[k] = ms / steps;
    if (first || ms < best_ms) {
      best = k;
      best_ms = ms;
      first = false;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r) {
    (void)tgks_batch_set_tile(b, old);
    return r;
  }
  if (chosen) *chosen = best;
  return tgks_batch_set_tile(b, best);
}

}  // extern "C"
