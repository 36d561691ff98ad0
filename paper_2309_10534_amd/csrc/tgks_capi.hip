// tgks_capi.hip -- C ABI of the TENO-D GKS library (declared in include/tgks.h).
//
// A context owns the device work buffers of one grid: the intermediate state
// W* and the accumulator P of the S2O4 step (Sec. 2.2), a ping-pong state for
// tgks_run, the per-direction face flux arrays, the 3-D normal
// reconstruction buffer, CFL partial minima, a device clock {t, dt} and the
// failure counter.  All launches go to the context's stream.
#include "tgks_internal.hpp"

using namespace tgks;

#define LAUNCH(kern, grid, block, args) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, args)

// face fluxes of one stage in every direction
int launch_faces(tgks_ctx* c, const double* W, const double* dt, int stage, uint8_t* flags) {
  const int D = c->g.D;
  if (c->p.scheme != TGKS_SCHEME_TENO_D) {
    const bool fl = flags != nullptr && stage == 1;
    StageArgs a[2];
    for (int ax = 0; ax < D; ++ax) {
      a[ax] = stage_args(c, W, ax, dt);
      if (fl) {
        a[ax].nflags = flags;
        long long off = (long long)D * c->nc * c->ncell;
        for (int d = 0; d < ax; ++d) off += 4LL * c->nc * c->nface[d];
        a[ax].tflags = D == 2 ? flags + off : nullptr;
      }
    }
    switch (c->p.scheme) {
      case TGKS_SCHEME_WENO_AO:
        return launch_scheme_faces<SCHEME_WENO_AO>(c, a, stage, fl);
      case TGKS_SCHEME_TENO5:
        return launch_scheme_faces<SCHEME_TENO5>(c, a, stage, fl);
      default:
        return launch_scheme_faces<SCHEME_WENO_Z>(c, a, stage, fl);
    }
  }
  if (D == 2) {
    // both directions in one launch (timed as kind 0)
    const bool fl = flags != nullptr && stage == 1;
    StageArgs a[2];
    for (int ax = 0; ax < 2; ++ax) {
      a[ax] = stage_args(c, W, ax, dt);
      if (fl) {
        a[ax].nflags = flags;
        long long off = (long long)D * c->nc * c->ncell;
        for (int d = 0; d < ax; ++d) off += 4LL * c->nc * c->nface[d];
        a[ax].tflags = flags + off;
      }
    }
    Timer tm(c, 0);
    launch_face2d_xy_any(c, a[0], a[1], stage, fl);
    HIPCHK(hipGetLastError());
    return TGKS_OK;
  }
  for (int ax = 0; ax < D; ++ax) {
    StageArgs a = stage_args(c, W, ax, dt);
    const bool fl = flags != nullptr && stage == 1;
    if (fl) {
      a.nflags = flags;
      if (D == 3) {
        // tangential flags of 3-D faces: 16 nc planes per direction
        long long off = (long long)D * c->nc * c->ncell;
        for (int d = 0; d < ax; ++d) off += 16LL * c->nc * c->nface[d];
        a.tflags = flags + off;
      }
    }
    if (D == 1) {
      Timer tm(c, 0);
      dim3 grid((unsigned)((c->g.n[0] + 1 + 255) / 256));
#define F1(CH, EX)                                                                  \
  if (stage == 1) {                                                                 \
    if (fl) {                                                                       \
      if (c->ns) LAUNCH((face1d_kernel<1, true, true, CH, EX>), grid, dim3(256), a);  \
      else LAUNCH((face1d_kernel<1, false, true, CH, EX>), grid, dim3(256), a);       \
    } else {                                                                        \
      if (c->ns) LAUNCH((face1d_kernel<1, true, false, CH, EX>), grid, dim3(256), a); \
      else LAUNCH((face1d_kernel<1, false, false, CH, EX>), grid, dim3(256), a);      \
    }                                                                               \
  } else {                                                                          \
    if (c->ns) LAUNCH((face1d_kernel<2, true, false, CH, EX>), grid, dim3(256), a);   \
    else LAUNCH((face1d_kernel<2, false, false, CH, EX>), grid, dim3(256), a);        \
  }
      const bool ch = c->p.recon == TGKS_RECON_CHARACTERISTIC;
      if (ch && c->ex) {
        F1(true, true)
      } else if (ch) {
        F1(true, false)
      } else if (c->ex) {
        F1(false, true)
      } else {
        F1(false, false)
      }
#undef F1
    } else if (D == 2) {
      Timer tm(c, ax);
      launch_face2d_any(c, a, ax, stage, fl);
    } else {
      int r = ax == 0 ? launch_face3d_ax<0>(c, a, stage, fl)
                      : (ax == 1 ? launch_face3d_ax<1>(c, a, stage, fl) : launch_face3d_ax<2>(c, a, stage, fl));
      if (r) return r;
    }
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static UpdateArgs update_args(tgks_ctx* c, const double* W, double* o1, double* o2, const double* dt,
                              double* partial) {
  UpdateArgs u;
  u.g = c->g;
  u.W = W;
  u.out1 = o1;
  u.out2 = o2;
  for (int d = 0; d < 3; ++d) {
    u.FA[d] = c->FA[d];
    u.FB[d] = c->FB[d];
  }
  u.dt = dt;
  u.gamma = c->p.gamma;
  u.mu = c->p.mu;
  u.partial = partial;
  return u;
}

int launch_update(tgks_ctx* c, int stage, const double* W, double* o1, double* o2, const double* dt,
                         bool cfl) {
  UpdateArgs u = update_args(c, W, o1, o2, dt, c->partial);
  dim3 grid((unsigned)c->nblk);
  Timer tm(c, stage == 1 ? 4 : 5);
#define UPD(DV)                                                                 \
  if (stage == 1) LAUNCH((update_kernel<DV, 1, false>), grid, dim3(256), u);    \
  else if (cfl) LAUNCH((update_kernel<DV, 2, true>), grid, dim3(256), u);       \
  else LAUNCH((update_kernel<DV, 2, false>), grid, dim3(256), u);
  if (c->g.D == 1) {
    UPD(1)
  } else if (c->g.D == 2) {
    UPD(2)
  } else {
    UPD(3)
  }
#undef UPD
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static int launch_cfl_partial(tgks_ctx* c, const double* W) {
  Timer tm(c, 6);
  dim3 grid((unsigned)c->nblk);
  if (c->g.D == 1)
    hipLaunchKernelGGL((cfl_partial_kernel<1>), grid, dim3(256), 0, c->stream, c->g, W, c->p.gamma, c->p.mu, c->partial);
  else if (c->g.D == 2)
    hipLaunchKernelGGL((cfl_partial_kernel<2>), grid, dim3(256), 0, c->stream, c->g, W, c->p.gamma, c->p.mu, c->partial);
  else
    hipLaunchKernelGGL((cfl_partial_kernel<3>), grid, dim3(256), 0, c->stream, c->g, W, c->p.gamma, c->p.mu, c->partial);
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

static int launch_finalize(tgks_ctx* c, double cfl, double t_in, double t_end, double* clock, double* dt_out,
                           int mode) {
  Timer tm(c, 6);
  hipLaunchKernelGGL(cfl_finalize_kernel, dim3(1), dim3(256), 0, c->stream, c->partial, c->nblk, cfl, t_in, t_end,
                     clock, dt_out, mode);
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

// one S2O4 step W -> out, dt read from dt_dev
int do_step(tgks_ctx* c, const double* W, double* out, const double* dt, uint8_t* flags, bool cfl) {
  int r;
  if ((r = launch_faces(c, W, dt, 1, flags))) return r;
  if ((r = launch_update(c, 1, W, c->Ws, c->P, dt, false))) return r;
  if ((r = launch_faces(c, c->Ws, dt, 2, nullptr))) return r;
  if ((r = launch_update(c, 2, c->P, out, nullptr, dt, cfl))) return r;
  return TGKS_OK;
}

static void free_ctx(tgks_ctx* c) {
  if (!c) return;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  (void)hipFree(c->Ws);
  (void)hipFree(c->P);
  (void)hipFree(c->W2);
  for (int d = 0; d < 3; ++d) {
    (void)hipFree(c->FA[d]);
    (void)hipFree(c->FB[d]);
  }
  (void)hipFree(c->R);
  (void)hipFree(c->partial);
  (void)hipFree(c->clock);
  (void)hipFree(c->fail);
  (void)hipFree(c->aGB);
  (void)hipFree(c->aTF);
  (void)hipFree(c->aNRB);
  (void)hipFree(c->aNF);
  (void)hipFree(c->aWsb);
  for (int k = 0; k < NKIND; ++k)
    for (auto& e : c->ev[k]) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  delete c;
}


extern "C" {

int tgks_params_default(tgks_params* p, int32_t ndim) {
  if (!p || ndim < 1 || ndim > 3) return TGKS_EINVAL;
  memset(p, 0, sizeof(*p));
  p->ndim = ndim;
  for (int d = 0; d < 3; ++d) {
    p->n[d] = 1;
    p->dx[d] = 1.0;
    p->bc_lo[d] = p->bc_hi[d] = TGKS_BC_TRANSMISSIVE;
  }
  p->gamma = 1.4;
  p->mu = 0.0;
  p->prandtl = 1.0;
  p->tau_mode = TGKS_TAU_INVISCID;
  p->c1 = 0.01;
  p->c2 = 1.0;
  p->ct1 = p->ct1_tan = 1e-7;
  p->ct2 = p->ct2_tan = 1e-5;
  p->eps = 1e-40;
  p->q = 7;
  p->scheme = TGKS_SCHEME_TENO_D;
  p->d_hi = p->d_lo = 0.85;
  p->eps_w = 1e-8;
  return TGKS_OK;
}

}  // extern "C"

// host-side description of a grid (no device memory): geometry, flux and
// selection constants
void init_ctx_host(tgks_ctx* c, const tgks_params* p, void* stream) {
  c->p = *p;
  c->pb = prescribed_of(p);
  c->ex = c->pb.on || p->fallback;
  c->stream = (hipStream_t)stream;
  const int D = p->ndim;
  c->nc = D + 2;
  Geom& g = c->g;
  g.D = D;
  g.ncell = 1;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = d < D ? p->n[d] : 1;
    g.dx[d] = d < D ? p->dx[d] : 1.0;
    g.bclo[d] = p->bc_lo[d];
    g.bchi[d] = p->bc_hi[d];
    g.ncell *= g.n[d];
  }
  c->ncell = g.ncell;
  const double N = 2.0 / (p->gamma - 1.0);
  c->fc.N = N;
  c->fc.K = N - D;
  c->fc.mu = p->mu;
  c->ns = p->mu > 0.0 && p->prandtl != 1.0;
  c->fc.pr_fix = c->ns ? 1.0 / p->prandtl - 1.0 : 0.0;
  c->fc.c1 = p->c1;
  c->fc.c2 = p->c2;
  c->fc.tau_mode = p->tau_mode;
  c->tn = teno_cfg(p->ct1, p->ct2, p->eps, p->q);
  c->tt = teno_cfg(p->ct1_tan, p->ct2_tan, p->eps, p->q);
  c->sc = {p->ct1, p->eps, p->q, p->d_hi, p->d_lo, p->eps_w};
  for (int d = 0; d < 3; ++d) {
    long long nf = 1;
    for (int e = 0; e < 3; ++e) nf *= (long long)(g.n[e] + (e == d));
    c->nface[d] = d < D ? nf : 0;
  }
  c->nblk = (int)((g.ncell + 255) / 256);
}

extern "C" {

int tgks_create(const tgks_params* p, void* stream, tgks_ctx** out) {
  if (!out || check_params(p)) return TGKS_EINVAL;
  *out = nullptr;
  tgks_ctx* c = new (std::nothrow) tgks_ctx();
  if (!c) return TGKS_EHIP;
  init_ctx_host(c, p, stream);
  const int D = p->ndim;
  const Geom& g = c->g;
  const size_t state = (size_t)c->nc * g.ncell * sizeof(double);
  bool ok = hipMalloc(&c->Ws, state) == hipSuccess && hipMalloc(&c->P, state) == hipSuccess &&
            hipMalloc(&c->W2, state) == hipSuccess;
  for (int d = 0; d < D && ok; ++d)
    ok = hipMalloc(&c->FA[d], (size_t)c->nc * c->nface[d] * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->FB[d], (size_t)c->nc * c->nface[d] * sizeof(double)) == hipSuccess;
  if (ok && D == 3) {
    long long mx = 0;
    for (int d = 0; d < 3; ++d) {
      long long nr = 1;
      for (int e = 0; e < 3; ++e) nr *= (long long)(g.n[e] + 2 * (e == d));
      mx = nr > mx ? nr : mx;
    }
    ok = hipMalloc(&c->R, (size_t)mx * 4 * 5 * sizeof(double)) == hipSuccess;
  }
  if (ok)
    ok = hipMalloc(&c->partial, (size_t)c->nblk * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->clock, 4 * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->fail, 2 * sizeof(unsigned long long)) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(256), 0, c->stream, c->fail, 2);
    ok = hipGetLastError() == hipSuccess;
  }
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) {
    free_ctx(c);
    return TGKS_EHIP;
  }
  *out = c;
  return TGKS_OK;
}

int tgks_destroy(tgks_ctx* c) {
  if (!c) return TGKS_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  return TGKS_OK;
}

int tgks_set_stream(tgks_ctx* c, void* stream) {
  if (!c) return TGKS_EINVAL;
  c->stream = (hipStream_t)stream;
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_steps = -1;
  }
  return TGKS_OK;
}

int64_t tgks_state_size(const tgks_ctx* c) { return c ? (int64_t)c->nc * c->ncell : TGKS_EINVAL; }

int64_t tgks_flag_bytes(const tgks_ctx* c) {
  if (!c) return TGKS_EINVAL;
  int64_t nb = (int64_t)c->g.D * c->nc * c->ncell;
  if (c->g.D == 2) nb += 4LL * c->nc * (c->nface[0] + c->nface[1]);
  if (c->g.D == 3) nb += 16LL * c->nc * (c->nface[0] + c->nface[1] + c->nface[2]);
  return nb;
}

int tgks_cfl_dt(tgks_ctx* c, const double* W, double cfl, double t, double t_end, double* dt_dev) {
  if (!c || !W || !dt_dev || !(cfl > 0.0)) return TGKS_EINVAL;
  int r;
  if ((r = launch_cfl_partial(c, W))) return r;
  return launch_finalize(c, cfl, t, t_end, nullptr, dt_dev, 0);
}

int tgks_step(tgks_ctx* c, const double* W_in, double* W_out, const double* dt_dev, uint8_t* flags,
              double* W_star) {
  if (!c || !W_in || !W_out || !dt_dev || W_in == W_out) return TGKS_EINVAL;
  int r = do_step(c, W_in, W_out, dt_dev, flags, false);
  if (r) return r;
  if (W_star)
    HIPCHK(hipMemcpyAsync(W_star, c->Ws, (size_t)c->nc * c->ncell * sizeof(double), hipMemcpyDeviceToDevice,
                          c->stream));
  return TGKS_OK;
}

static int enqueue_run(tgks_ctx* c, double* W, int n_steps, double cfl, double t_end, double fixed_dt,
                       double* time_dev) {
  int r = 0;
  const bool use_cfl = cfl > 0.0;
  if (use_cfl) {
    if ((r = launch_cfl_partial(c, W))) return r;
    if ((r = launch_finalize(c, cfl, 0.0, t_end, c->clock, nullptr, 0))) return r;
  } else {
    hipLaunchKernelGGL(set_clock_kernel, dim3(1), dim3(1), 0, c->stream, c->clock, 0.0, fixed_dt);
    HIPCHK(hipGetLastError());
  }
  double* src = W;
  double* dst = c->W2;
  c->tclk = c->clock;  // the state of each step is that of time t0 + clock[0]
  for (int s = 0; s < n_steps; ++s) {
    if ((r = do_step(c, src, dst, c->clock + 1, nullptr, use_cfl))) break;
    if ((r = launch_finalize(c, cfl, 0.0, t_end, c->clock, nullptr, use_cfl ? 1 : 2))) break;
    double* t = src;
    src = dst;
    dst = t;
  }
  c->tclk = nullptr;
  if (r) return r;
  if (src != W)
    HIPCHK(hipMemcpyAsync(W, src, (size_t)c->nc * c->ncell * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (time_dev)
    HIPCHK(hipMemcpyAsync(time_dev, c->clock, 2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return TGKS_OK;
}

int tgks_run(tgks_ctx* c, double* W, int32_t n_steps, double cfl, double t_end, double fixed_dt, double* time_dev,
             int32_t use_graph) {
  if (!c || !W || n_steps < 0) return TGKS_EINVAL;
  if (!(cfl > 0.0) && !(fixed_dt > 0.0)) return TGKS_EINVAL;
  if (!use_graph || c->timing) return enqueue_run(c, W, n_steps, cfl, t_end, fixed_dt, time_dev);
  const bool same = c->gexec && c->g_steps == n_steps && c->g_cfl == cfl && c->g_tend == t_end &&
                    c->g_fixed == fixed_dt && c->g_W == W && c->g_time == time_dev &&
                    (!c->pb.on || c->g_t0 == c->t0);
  if (!same) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      (void)hipGraphDestroy(c->graph);
      c->gexec = nullptr;
      c->graph = nullptr;
    }
    if (c->stream == nullptr) return enqueue_run(c, W, n_steps, cfl, t_end, fixed_dt, time_dev);
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int r = enqueue_run(c, W, n_steps, cfl, t_end, fixed_dt, time_dev);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (r) {
      if (gr) (void)hipGraphDestroy(gr);
      return r;
    }
    if (e != hipSuccess) {
      fprintf(stderr, "tgks: graph capture failed: %s\n", hipGetErrorString(e));
      return TGKS_EHIP;
    }
    c->graph = gr;
    HIPCHK(hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0));
    c->g_steps = n_steps;
    c->g_cfl = cfl;
    c->g_tend = t_end;
    c->g_fixed = fixed_dt;
    c->g_W = W;
    c->g_time = time_dev;
    c->g_t0 = c->t0;
  }
  HIPCHK(hipGraphLaunch(c->gexec, c->stream));
  return TGKS_OK;
}

int tgks_fallback_count(tgks_ctx* c, int64_t* count) {
  if (!c || !count) return TGKS_EINVAL;
  unsigned long long h = 0;
  HIPCHK(hipMemcpyAsync(&h, c->fail + 1, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *count = (int64_t)h;
  return TGKS_OK;
}

int tgks_set_time(tgks_ctx* c, double t0) {
  if (!c || !std::isfinite(t0)) return TGKS_EINVAL;
  c->t0 = t0;
  return TGKS_OK;
}

int tgks_status(tgks_ctx* c, int64_t* failures) {
  if (!c || !failures) return TGKS_EINVAL;
  unsigned long long h = 0;
  HIPCHK(hipMemcpyAsync(&h, c->fail, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *failures = (int64_t)h;
  return TGKS_OK;
}

int tgks_reset_status(tgks_ctx* c) {
  if (!c) return TGKS_EINVAL;
  hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(256), 0, c->stream, c->fail, 2);
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

int tgks_timing(tgks_ctx* c, int32_t enable) {
  if (!c) return TGKS_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < NKIND; ++k) {
    for (auto& e : c->ev[k]) {
      c->pool.push_back(e.a);
      c->pool.push_back(e.b);
    }
    c->ev[k].clear();
  }
  c->timing = enable != 0;
  return TGKS_OK;
}

int tgks_kernel_time(tgks_ctx* c, int32_t kind, double* ms, int64_t* launches) {
  if (!c || kind < 0 || kind >= NKIND || !ms || !launches) return TGKS_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (auto& e : c->ev[kind]) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e.a, e.b));
    s += t;
  }
  *ms = s;
  *launches = (int64_t)c->ev[kind].size();
  return TGKS_OK;
}

}  // extern "C"

namespace {
template <int D>
int host_flux(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl, const double* dWr,
              double dt, double* F) {
  constexpr int NC = D + 2;
  FluxCfg fc;
  const double N = 2.0 / (p->gamma - 1.0);
  fc.N = N;
  fc.K = N - D;
  fc.mu = p->mu;
  const bool ns = p->mu > 0.0 && p->prandtl != 1.0;
  fc.pr_fix = ns ? 1.0 / p->prandtl - 1.0 : 0.0;
  fc.c1 = p->c1;
  fc.c2 = p->c2;
  fc.tau_mode = p->tau_mode;
  double l[NC], r[NC], dl[D][NC], dr[D][NC], Fdt[NC], Fh[NC];
  for (int q = 0; q < NC; ++q) {
    l[q] = Wl[q];
    r[q] = Wr[q];
    for (int d = 0; d < D; ++d) {
      dl[d][q] = dWl[d * NC + q];
      dr[d][q] = dWr[d * NC + q];
    }
  }
  const bool ok = ns ? gp_flux<D, true>(l, r, dl, dr, fc, dt, Fdt, Fh) : gp_flux<D, false>(l, r, dl, dr, fc, dt, Fdt, Fh);
  for (int q = 0; q < NC; ++q) {
    F[q] = Fdt[q];
    F[NC + q] = Fh[q];
  }
  return ok ? 0 : 1;
}
}  // namespace

extern "C" {

int tgks_teno_flag_host(const tgks_params* p, const double* Q, int32_t fast) {
  if (check_params(p) || !Q) return TGKS_EINVAL;
  const TenoCfg c = teno_cfg(p->ct1, p->ct2, p->eps, p->q);
  if (fast < 0 || fast > 2) return TGKS_EINVAL;
  return (int)(fast == 1 ? teno_flag<SEL_RATIO>(Q, c)
                         : (fast == 2 ? teno_flag<SEL_FILTER>(Q, c) : teno_flag<SEL_EXACT>(Q, c)));
}

double tgks_erfc_host(double x) { return erfc_exp(x, exp(-x * x)); }

int tgks_gp_flux_host(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl, const double* dWr,
                      double dt, double* F) {
  if (check_params(p) || !Wl || !Wr || !dWl || !dWr || !F) return TGKS_EINVAL;
  if (p->ndim == 1) return host_flux<1>(p, Wl, Wr, dWl, dWr, dt, F);
  if (p->ndim == 2) return host_flux<2>(p, Wl, Wr, dWl, dWr, dt, F);
  return host_flux<3>(p, Wl, Wr, dWl, dWr, dt, F);
}

int tgks_set_tile(tgks_ctx* c, int32_t tile) {
  if (!c || tile < -1 || tile >= NTILE2) return TGKS_EINVAL;
  int t = tile < 0 ? 0 : tile;
  if (c->g.D == 2 && (c->p.recon == TGKS_RECON_CHARACTERISTIC || c->ex)) t = CHAR_TILE2;
  if (t != c->tile2 && c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->g_steps = -1;
  }
  c->tile2 = t;
  return TGKS_OK;
}

int tgks_tune(tgks_ctx* c, const double* W, int32_t steps, int32_t* chosen, float* ms_per_variant) {
  if (!c || !W || steps < 1) return TGKS_EINVAL;
  const int nvar = c->g.D == 2 ? NTILE2 : 1;
  int r;
  // dt of W into the clock (no clipping)
  if ((r = launch_cfl_partial(c, W))) return r;
  if ((r = launch_finalize(c, 0.5, 0.0, 0.0, c->clock, nullptr, 0))) return r;
  const bool timing = c->timing;
  c->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.f;
  const int old = c->tile2;
  const bool char2 = c->g.D == 2 && (c->p.recon == TGKS_RECON_CHARACTERISTIC || c->ex);
  bool first = true;
  for (int k = 0; k < nvar; ++k) {
    if (char2 && k != CHAR_TILE2) {  // one tile shape on the characteristic / extras path
      if (ms_per_variant) ms_per_variant[k] = 0.f;
      continue;
    }
    c->tile2 = k;
    if ((r = do_step(c, W, c->W2, c->clock + 1, nullptr, false))) break;  // warm-up
    HIPCHK(hipEventRecord(e0, c->stream));
    for (int s = 0; s < steps && !r; ++s) r = do_step(c, W, c->W2, c->clock + 1, nullptr, false);
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms_per_variant) ms_per_variant[k] = ms / steps;
    if (first || ms < best_ms) {
      best = k;
      best_ms = ms;
      first = false;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = timing;
  c->tile2 = old;
  if (r) return r;
  if (chosen) *chosen = best;
  return tgks_set_tile(c, best);
}

}  // extern "C"
