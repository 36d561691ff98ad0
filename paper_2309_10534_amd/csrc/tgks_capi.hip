// tgks_capi.hip -- C ABI of the TENO-D GKS library (declared in include/tgks.h).
//
// A context owns the device work buffers of one grid: the intermediate state
// W* and the accumulator P of the S2O4 step (Sec. 2.2), a ping-pong state for
// tgks_run, the per-direction face flux arrays, the 3-D normal
// reconstruction buffer, CFL partial minima, a device clock {t, dt} and the
// failure counter.  All launches go to the context's stream.
#include "tgks_internal.hpp"
#include "tgks_opcount.hpp"

using namespace tgks;

#define LAUNCH(kern, grid, block, args) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, args)

// face fluxes of one stage in every direction
int launch_faces(tgks_ctx* c, const double* W, const double* dt, int stage, uint8_t* flags) {
  const int D = c->g.D;
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
      if (D == 2) {
        long long off = (long long)D * c->nc * c->ncell;
        for (int d = 0; d < ax; ++d) off += 4LL * c->nc * c->nface[d];
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
      int ext[3] = {c->g.n[0], c->g.n[1], c->g.n[2]};
      ext[ax] += 2;
      const long long nr = (long long)ext[0] * ext[1] * ext[2];
      {
        Timer tm(c, 3);
        dim3 grid((unsigned)((nr * 5 + 255) / 256));
#define R3(AXV)                                                                   \
  if (fl) LAUNCH((recon3d_kernel<AXV, true>), grid, dim3(256), a);                \
  else LAUNCH((recon3d_kernel<AXV, false>), grid, dim3(256), a);
        if (ax == 0) {
          R3(0)
        } else if (ax == 1) {
          R3(1)
        } else {
          R3(2)
        }
#undef R3
      }
      {
        Timer tm(c, ax);
        const int n1 = c->g.n[(ax + 1) % 3], n2 = c->g.n[(ax + 2) % 3];
        const long long nbl = (long long)(c->g.n[ax] + 1) * ((n1 + B3_1 - 1) / B3_1) * ((n2 + B3_2 - 1) / B3_2);
        dim3 grid((unsigned)(8 * ((nbl + 7) / 8)));
        const dim3 blk3(L3 * B3_1 * B3_2);
#define F3(AXV, EX)                                                                   \
  if (stage == 1) {                                                                   \
    if (c->ns) LAUNCH((face3d_kernel<AXV, 1, true, EX>), grid, blk3, a);              \
    else LAUNCH((face3d_kernel<AXV, 1, false, EX>), grid, blk3, a);                   \
  } else {                                                                            \
    if (c->ns) LAUNCH((face3d_kernel<AXV, 2, true, EX>), grid, blk3, a);              \
    else LAUNCH((face3d_kernel<AXV, 2, false, EX>), grid, blk3, a);                   \
  }
        if (c->ex) {  // the first-order fallback (3-D grids have no prescribed sides)
          if (ax == 0) {
            F3(0, true)
          } else if (ax == 1) {
            F3(1, true)
          } else {
            F3(2, true)
          }
        } else if (ax == 0) {
          F3(0, false)
        } else if (ax == 1) {
          F3(1, false)
        } else {
          F3(2, false)
        }
#undef F3
      }
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
static int do_step(tgks_ctx* c, const double* W, double* out, const double* dt, uint8_t* flags, bool cfl) {
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

// ---------------------------------------------------------------------------
// Algorithmic operation counts: the kernels' per-cell and per-face sequences
// evaluated on the host with the counting scalar type, on smooth data (the
// large-stencil branch of every selection).
// ---------------------------------------------------------------------------
namespace {

using tgks_opcount::F;

F smooth(int c, double x, double y) {
  // conservative components of a smooth state (rho, rho u, rho v, rho w, rho E),
  // each a distinct input of the dataflow graph
  const double rho = 1.0 + 0.1 * std::sin(0.7 * x + 0.3 * y), u = 0.3, v = -0.2, w = 0.1, p = 1.0;
  switch (c) {
    case 0: return F::input(rho);
    case 1: return F::input(rho * u);
    case 2: return F::input(rho * v);
    case 3: return F::input(rho * w);
    default: return F::input(p / 0.4 + 0.5 * rho * (u * u + v * v + w * w));
  }
}

long long count_normal(const tgks_ctx* c) {
  F Q[5], o[4];
  tgks_opcount::graph().reset();
  for (int r = 0; r < 5; ++r) Q[r] = smooth(0, 0.1 * r, 0.0);
  const unsigned fl = teno_flag(Q, c->tn);
  teno_face(Q, fl, o);
  const F idn(1.0 / c->g.dx[0]);
  F s1 = o[1] * idn, s3 = o[3] * idn;
  (void)s1;
  (void)s3;
  return tgks_opcount::tally().total();
}

template <int D, bool NS>
long long count_face(const tgks_ctx* c, int stage, tgks_opcount::Tally* detail) {
  constexpr int NC = D + 2;
  const int NG = D == 1 ? 1 : (D == 2 ? 2 : 4);
  F Wg[4][2][NC], Dg[4][2][D][NC];
  tgks_opcount::graph().reset();
  for (int m = 0; m < NG; ++m)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < NC; ++q) {
        Wg[m][s][q] = smooth(q < D + 1 ? q : 4, 0.05 * s, 0.1 * m);
        for (int d = 0; d < D; ++d) Dg[m][s][d][q] = F::input(0.01 * (q + 1) * (d + 1));
      }
  if (D == 2) {
    // tangential reconstruction: per side and component, two selections, two
    // Gauss-point evaluations and the slope scaling
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < NC; ++q) {
        F Qw[5], Qn[5], v[2], dv[2], vn[2], dvn[2];
        for (int r = 0; r < 5; ++r) {
          Qw[r] = smooth(q < 3 ? q : 4, 0.1 * r, 0.0);
          Qn[r] = F::input(0.01 * r);
        }
        teno_gauss(Qw, teno_flag(Qw, c->tt), v, dv);
        teno_gauss(Qn, teno_flag(Qn, c->tt), vn, dvn);
        for (int m = 0; m < 2; ++m) dv[m] = dv[m] * F(1.0 / c->g.dx[1]);
      }
  } else if (D == 3) {
    // per side and component: the sweep-1 reconstruction of (W, W_n) along
    // t1 of this face's own line (the lines of the four neighbouring faces
    // along t2 are their work, inputs here), then per t1 Gauss point three
    // sweep-2 reconstructions along t2
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < NC; ++q) {
        F S1w[2][5], S1d[2][5], S1n[2][5];
        for (int r2 = 0; r2 < 5; ++r2) {
          if (r2 == 2) {
            F Qw[5], Qn[5], v[2], dv[2], vn[2], dvn[2];
            for (int r = 0; r < 5; ++r) {
              Qw[r] = smooth(q, 0.1 * r, 0.1 * r2);
              Qn[r] = F::input(0.01 * r);
            }
            teno_gauss(Qw, teno_flag(Qw, c->tt), v, dv);
            teno_gauss(Qn, teno_flag(Qn, c->tt), vn, dvn);
            for (int m1 = 0; m1 < 2; ++m1) {
              S1w[m1][r2] = v[m1];
              S1d[m1][r2] = dv[m1] * F(1.0 / c->g.dx[1]);
              S1n[m1][r2] = vn[m1];
            }
          } else {
            for (int m1 = 0; m1 < 2; ++m1) {
              S1w[m1][r2] = smooth(q, 0.1 * m1, 0.1 * r2);
              S1d[m1][r2] = F::input(0.02 * (r2 + 1) + 0.01 * m1);
              S1n[m1][r2] = F::input(0.03 * (r2 + 1) + 0.01 * m1);
            }
          }
        }
        for (int m1 = 0; m1 < 2; ++m1) {
          F v[2], dv[2], x[2], dx_[2];
          teno_gauss(S1w[m1], teno_flag(S1w[m1], c->tt), v, dv);
          for (int m2 = 0; m2 < 2; ++m2) dv[m2] = dv[m2] * F(1.0 / c->g.dx[2]);
          teno_gauss(S1d[m1], teno_flag(S1d[m1], c->tt), x, dx_);
          teno_gauss(S1n[m1], teno_flag(S1n[m1], c->tt), x, dx_);
        }
      }
  }
  FluxCfg fc = c->fc;
  const F dt(1e-3);
  F A[NC], B[NC];
  for (int q = 0; q < NC; ++q) A[q] = B[q] = F(0.0);
  const double w = 1.0 / NG;
  for (int m = 0; m < NG; ++m) {
    F Fdt[NC], Fh[NC];
    gp_flux<D, NS>(Wg[m][0], Wg[m][1], Dg[m][0], Dg[m][1], fc, dt, Fdt, Fh);
    for (int q = 0; q < NC; ++q) {
      if (stage == 1) {
        A[q] += F(w) * Fh[q];
        B[q] += F(w) * (F(8.0 / 3.0) * Fh[q] - F(1.0 / 3.0) * Fdt[q]);
      } else {
        A[q] += F(w) * (F(4.0 / 3.0) * Fdt[q] - F(8.0 / 3.0) * Fh[q]);
      }
    }
  }
  if (detail) *detail = tgks_opcount::tally();
  return tgks_opcount::tally().total();
}

// Characteristic variables: the face's own normal reconstruction (basis at
// the face mean state, projection of the six cells, both sides' selections,
// back-projection) belongs to the face; in 2-D the faces of the tangential
// stencil are their own work (inputs here), followed by the tangential
// basis, projections, selections and back-projections of both sides and the
// two Gauss-point fluxes.
template <int D, bool NS>
long long count_face_char(const tgks_ctx* c, int stage, tgks_opcount::Tally* detail) {
  constexpr int NC = D + 2;
  constexpr int NG = D == 1 ? 1 : 2;
  tgks_opcount::graph().reset();
  F C[6][NC];
  for (int r = 0; r < 6; ++r)
    for (int q = 0; q < NC; ++q) C[r][q] = smooth(q < D + 1 ? q : 4, 0.1 * r, 0.0);
  F vl[NC], sl[NC], vr[NC], sr[NC];
  unsigned fr[NC];
  char_recon_face<D>(c->p.gamma, C, c->tn, 1.0 / c->g.dx[0], vl, sl, vr, sr, fr);
  F Wg[2][2][NC], Dg[2][2][D][NC];
  if (D == 1) {
    for (int q = 0; q < NC; ++q) {
      Wg[0][0][q] = vl[q];
      Wg[0][1][q] = vr[q];
      Dg[0][0][0][q] = sl[q];
      Dg[0][1][0][q] = sr[q];
    }
  } else {
    F Wb[NC], L[NC][NC], R[NC][NC];
    for (int q = 0; q < NC; ++q) Wb[q] = F(0.5) * (C[2][q] + C[3][q]);
    char_basis<D, D - 1>(c->p.gamma, Wb, L, R);
    for (int s = 0; s < 2; ++s) {
      F X[5][NC], Xn[5][NC];
      for (int r = 0; r < 5; ++r)
        for (int q = 0; q < NC; ++q) {
          X[r][q] = r == 2 ? (s == 0 ? vl[q] : vr[q]) : smooth(q < D + 1 ? q : 4, 0.1 * r, 0.05 * s);
          Xn[r][q] = r == 2 ? (s == 0 ? sl[q] : sr[q]) : F::input(0.01 * (r + 1) * (q + 1));
        }
      F aV[NC][2], aD[NC][2], aN[NC][2];
      for (int k = 0; k < NC; ++k) {
        F Qw[5], Qn[5], v[2], dv[2], vn[2], dvn[2];
        for (int r = 0; r < 5; ++r) {
          Qw[r] = char_dot<NC>(L[k], X[r]);
          Qn[r] = char_dot<NC>(L[k], Xn[r]);
        }
        teno_gauss(Qw, teno_flag(Qw, c->tt), v, dv);
        teno_gauss(Qn, teno_flag(Qn, c->tt), vn, dvn);
        for (int q = 0; q < NC; ++q)
          for (int g = 0; g < 2; ++g) {
            aV[q][g] = k == 0 ? R[q][k] * v[g] : aV[q][g] + R[q][k] * v[g];
            aD[q][g] = k == 0 ? R[q][k] * dv[g] : aD[q][g] + R[q][k] * dv[g];
            aN[q][g] = k == 0 ? R[q][k] * vn[g] : aN[q][g] + R[q][k] * vn[g];
          }
      }
      for (int g = 0; g < 2; ++g)
        for (int q = 0; q < NC; ++q) {
          Wg[g][s][q] = aV[q][g];
          Dg[g][s][0][q] = aN[q][g];
          Dg[g][s][D - 1][q] = aD[q][g] * F(1.0 / c->g.dx[1]);
        }
    }
  }
  FluxCfg fc = c->fc;
  const F dt(1e-3);
  F A[NC], B[NC];
  for (int q = 0; q < NC; ++q) A[q] = B[q] = F(0.0);
  const double w = 1.0 / NG;
  for (int m = 0; m < NG; ++m) {
    F Fdt[NC], Fh[NC];
    gp_flux<D, NS>(Wg[m][0], Wg[m][1], Dg[m][0], Dg[m][1], fc, dt, Fdt, Fh);
    for (int q = 0; q < NC; ++q) {
      if (stage == 1) {
        A[q] += F(w) * Fh[q];
        B[q] += F(w) * (F(8.0 / 3.0) * Fh[q] - F(1.0 / 3.0) * Fdt[q]);
      } else {
        A[q] += F(w) * (F(4.0 / 3.0) * Fdt[q] - F(8.0 / 3.0) * Fh[q]);
      }
    }
  }
  if (detail) *detail = tgks_opcount::tally();
  return tgks_opcount::tally().total();
}

template <int D>
long long count_face_dispatch(const tgks_ctx* c, int stage, tgks_opcount::Tally* t) {
  if constexpr (D <= 2) {
    if (c->p.recon == TGKS_RECON_CHARACTERISTIC)
      return c->ns ? count_face_char<D, true>(c, stage, t) : count_face_char<D, false>(c, stage, t);
  }
  return c->ns ? count_face<D, true>(c, stage, t) : count_face<D, false>(c, stage, t);
}

}  // namespace

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
  return TGKS_OK;
}

int tgks_create(const tgks_params* p, void* stream, tgks_ctx** out) {
  if (!out || check_params(p)) return TGKS_EINVAL;
  *out = nullptr;
  tgks_ctx* c = new (std::nothrow) tgks_ctx();
  if (!c) return TGKS_EHIP;
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
  c->tn = {p->ct1, p->ct2, p->eps, p->q};
  c->tt = {p->ct1_tan, p->ct2_tan, p->eps, p->q};
  const size_t state = (size_t)c->nc * g.ncell * sizeof(double);
  bool ok = hipMalloc(&c->Ws, state) == hipSuccess && hipMalloc(&c->P, state) == hipSuccess &&
            hipMalloc(&c->W2, state) == hipSuccess;
  for (int d = 0; d < D && ok; ++d) {
    long long nf = 1;
    for (int e = 0; e < 3; ++e) nf *= (long long)(g.n[e] + (e == d));
    c->nface[d] = nf;
    ok = hipMalloc(&c->FA[d], (size_t)c->nc * nf * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->FB[d], (size_t)c->nc * nf * sizeof(double)) == hipSuccess;
  }
  if (ok && D == 3) {
    long long mx = 0;
    for (int d = 0; d < 3; ++d) {
      long long nr = 1;
      for (int e = 0; e < 3; ++e) nr *= (long long)(g.n[e] + 2 * (e == d));
      mx = nr > mx ? nr : mx;
    }
    ok = hipMalloc(&c->R, (size_t)mx * 4 * 5 * sizeof(double)) == hipSuccess;
  }
  c->nblk = (int)((g.ncell + 255) / 256);
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

int tgks_flop_counts(const tgks_params* p, double* out, int32_t nout) {
  if (!out || nout < 8 || check_params(p)) return TGKS_EINVAL;
  // a context-like description without device buffers
  tgks_ctx c;
  c.p = *p;
  const int D = p->ndim;
  c.nc = D + 2;
  c.g.D = D;
  for (int d = 0; d < 3; ++d) {
    c.g.n[d] = d < D ? p->n[d] : 1;
    c.g.dx[d] = d < D ? p->dx[d] : 1.0;
  }
  const double N = 2.0 / (p->gamma - 1.0);
  c.fc.N = N;
  c.fc.K = N - D;
  c.fc.mu = p->mu;
  c.ns = p->mu > 0.0 && p->prandtl != 1.0;
  c.fc.pr_fix = c.ns ? 1.0 / p->prandtl - 1.0 : 0.0;
  c.fc.c1 = p->c1;
  c.fc.c2 = p->c2;
  c.fc.tau_mode = p->tau_mode;
  c.tn = {p->ct1, p->ct2, p->eps, p->q};
  c.tt = {p->ct1_tan, p->ct2_tan, p->eps, p->q};
  tgks_opcount::Tally t1;
  long long f1, f2;
  if (D == 1) {
    f1 = count_face_dispatch<1>(&c, 1, &t1);
    f2 = count_face_dispatch<1>(&c, 2, nullptr);
  } else if (D == 2) {
    f1 = count_face_dispatch<2>(&c, 1, &t1);
    f2 = count_face_dispatch<2>(&c, 2, nullptr);
  } else {
    f1 = count_face_dispatch<3>(&c, 1, &t1);
    f2 = count_face_dispatch<3>(&c, 2, nullptr);
  }
  // characteristic variables: the normal reconstruction is part of the face work
  const long long nr = p->recon == TGKS_RECON_CHARACTERISTIC ? 0 : count_normal(&c);
  const int nc = D + 2;
  out[0] = (double)nr;                       // normal reconstruction, per cell, direction and component
  out[1] = (double)f1;                       // stage-1 face work beyond the normal reconstruction, per face
  out[2] = (double)f2;                       // stage-2 face work, per face
  out[3] = (double)(nc * D * 6);             // stage-1 update per cell: 2 states x D x (sub, div, sub)
  out[4] = (double)(nc * D * 3);             // stage-2 update per cell
  out[5] = (double)(t1.sqrt + t1.exp + t1.expm1 + t1.erfc);  // transcendentals per stage-1 face
  out[6] = (double)t1.div;                   // divisions per stage-1 face
  out[7] = (double)(D * 3 + 9);              // CFL limit per cell
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
