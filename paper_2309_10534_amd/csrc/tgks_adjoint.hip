// tgks_adjoint.hip -- reverse mode of one S2O4 step (include/tgks.h).
//
// With W* = W - sum_d D_d FA(W) / dx_d, P = W - sum_d D_d FB(W) / dx_d and
// W^{n+1} = P - sum_d D_d FA*(W*) / dx_d (the folded form of Sec. 2.2), the
// cotangent G of W^{n+1} gives
//   G* = (dFA*/dW*)^T D^T G                         (stage 2 at W*)
//   G_n = G + G* + (dFA/dW)^T D^T G* + (dFB/dW)^T D^T G   (stage 1 at W)
// with FA* = 4/3 F*(dt) - 8/3 F*(dt/2), FA = F(dt/2), FB = 8/3 F(dt/2) -
// 1/3 F(dt).  W* is recomputed with the forward kernels (bit-identical to
// the forward step, so every stencil selection is the forward's).
#include "tgks_adjoint_kernels.hpp"
#include "tgks_internal.hpp"

using namespace tgks;

static int ensure_adjoint_buffers(tgks_ctx* c) {
  if (c->aNRB) return TGKS_OK;
  const Geom& g = c->g;
  long long ne = 0, nf = 0;
  for (int ax = 0; ax < g.D; ++ax) {
    const long long e = g.D == 1 ? (long long)g.n[0] + 2 : (long long)(g.n[ax] + 2) * (g.n[1 - ax] + 4);
    ne = e > ne ? e : ne;
    nf = c->nface[ax] > nf ? c->nface[ax] : nf;
  }
  bool ok = hipMalloc(&c->aNRB, (size_t)c->nc * 4 * ne * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->aNF, (size_t)c->nc * ne) == hipSuccess &&
            hipMalloc(&c->aWsb, (size_t)c->nc * c->ncell * sizeof(double)) == hipSuccess;
  if (ok && g.D == 2)
    ok = hipMalloc(&c->aGB, (size_t)2 * c->nc * 6 * nf * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->aTF, (size_t)2 * 2 * c->nc * nf) == hipSuccess;
  if (!ok) {
    (void)hipFree(c->aNRB);
    (void)hipFree(c->aNF);
    (void)hipFree(c->aWsb);
    (void)hipFree(c->aGB);
    (void)hipFree(c->aTF);
    c->aNRB = c->aWsb = c->aGB = nullptr;
    c->aTF = c->aNF = nullptr;
    return TGKS_EHIP;
  }
  return TGKS_OK;
}

static AdjArgs adj_args(tgks_ctx* c, const double* W, const double* X, const double* Y, double cxdt, double cxh,
                        double cydt, double cyh, const double* dt) {
  AdjArgs a;
  a.g = c->g;
  a.fc = c->fc;
  a.tn = c->tn;
  a.tt = c->tt;
  a.W = W;
  a.X = X;
  a.Y = Y;
  a.cx_dt = cxdt;
  a.cx_h = cxh;
  a.cy_dt = cydt;
  a.cy_h = cyh;
  a.dt = dt;
  a.GB = c->aGB;
  a.TF = c->aTF;
  a.NRB = c->aNRB;
  a.NF = c->aNF;
  a.base0 = nullptr;
  a.base1 = nullptr;
  a.out = nullptr;
  return a;
}

#define ALAUNCH(kern, grid, block, args) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, args)

// reverse of the flux stage of direction ax at state W: out = base0 + base1 +
// (dF/dW)^T (face cotangents built from X, Y)
static int reverse_direction(tgks_ctx* c, AdjArgs a, int ax, const double* base0, const double* base1,
                             double* out) {
  const Geom& g = c->g;
  a.base0 = base0;
  a.base1 = base1;
  a.out = out;
  const int nc = c->nc;
  if (g.D == 1) {
    const dim3 grid((unsigned)((g.n[0] + 1 + 127) / 128));
    if (c->ns)
      ALAUNCH((adj_face1d_kernel<true>), grid, dim3(128), a);
    else
      ALAUNCH((adj_face1d_kernel<false>), grid, dim3(128), a);
    const dim3 gf((unsigned)(((g.n[0] + 2) * nc + 255) / 256));
    ALAUNCH((adj_nflags_kernel<1, 0>), gf, dim3(256), a);
    const dim3 gn((unsigned)((g.ncell * nc + 255) / 256));
    ALAUNCH((adj_normal_kernel<1, 0>), gn, dim3(256), a);
  } else {
    const int nN = g.n[ax], nT = g.n[1 - ax];
    const dim3 grid((unsigned)((nN + 1 + ATN - 1) / ATN), (unsigned)((nT + ATT - 1) / ATT));
    const long long ne = (long long)(nN + 2) * (nT + 4);
    const dim3 gt((unsigned)((ne * nc + 255) / 256));
    const dim3 gn((unsigned)((g.ncell * nc + 255) / 256));
    if (ax == 0) {
      if (c->ns)
        ALAUNCH((adj_face2d_kernel<0, true>), grid, dim3(2 * ATN * ATT), a);
      else
        ALAUNCH((adj_face2d_kernel<0, false>), grid, dim3(2 * ATN * ATT), a);
      ALAUNCH((adj_tan2d_kernel<0>), gt, dim3(256), a);
      ALAUNCH((adj_nflags_kernel<2, 0>), gt, dim3(256), a);
      ALAUNCH((adj_normal_kernel<2, 0>), gn, dim3(256), a);
    } else {
      if (c->ns)
        ALAUNCH((adj_face2d_kernel<1, true>), grid, dim3(2 * ATN * ATT), a);
      else
        ALAUNCH((adj_face2d_kernel<1, false>), grid, dim3(2 * ATN * ATT), a);
      ALAUNCH((adj_tan2d_kernel<1>), gt, dim3(256), a);
      ALAUNCH((adj_nflags_kernel<2, 1>), gt, dim3(256), a);
      ALAUNCH((adj_normal_kernel<2, 1>), gn, dim3(256), a);
    }
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}

namespace {
template <int D>
int host_flux_vjp(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl, const double* dWr,
                  double dt, const double* Fb, double* G) {
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
  double l[NC], r[NC], dl[D][NC], dr[D][NC], fdtb[NC], fhb[NC];
  double lb[NC], rb[NC], dlb[D][NC], drb[D][NC];
  for (int q = 0; q < NC; ++q) {
    l[q] = Wl[q];
    r[q] = Wr[q];
    fdtb[q] = Fb[q];
    fhb[q] = Fb[NC + q];
    for (int d = 0; d < D; ++d) {
      dl[d][q] = dWl[d * NC + q];
      dr[d][q] = dWr[d * NC + q];
    }
  }
  if (ns)
    gp_flux_vjp<D, true, double>(l, r, dl, dr, fc, dt, fdtb, fhb, lb, rb, dlb, drb);
  else
    gp_flux_vjp<D, false, double>(l, r, dl, dr, fc, dt, fdtb, fhb, lb, rb, dlb, drb);
  for (int q = 0; q < NC; ++q) {
    G[q] = lb[q];
    G[NC + q] = rb[q];
    for (int d = 0; d < D; ++d) {
      G[2 * NC + d * NC + q] = dlb[d][q];
      G[2 * NC + D * NC + d * NC + q] = drb[d][q];
    }
  }
  return TGKS_OK;
}
}  // namespace

extern "C" {

int tgks_gp_flux_vjp_host(const tgks_params* p, const double* Wl, const double* Wr, const double* dWl,
                          const double* dWr, double dt, const double* Fb, double* G) {
  if (check_params(p) || !Wl || !Wr || !dWl || !dWr || !Fb || !G) return TGKS_EINVAL;
  if (p->ndim == 1) return host_flux_vjp<1>(p, Wl, Wr, dWl, dWr, dt, Fb, G);
  if (p->ndim == 2) return host_flux_vjp<2>(p, Wl, Wr, dWl, dWr, dt, Fb, G);
  return host_flux_vjp<3>(p, Wl, Wr, dWl, dWr, dt, Fb, G);
}

int tgks_step_adjoint(tgks_ctx* c, const double* W_n, const double* W_star, const double* dt_dev,
                      const double* gW_out, double* gW_in) {
  if (!c || !W_n || !dt_dev || !gW_out || !gW_in || gW_out == gW_in) return TGKS_EINVAL;
  if (c->g.D > 2 || c->p.recon != TGKS_RECON_CONSERVATIVE || c->pb.on || c->p.fallback ||
      c->p.scheme != TGKS_SCHEME_TENO_D)
    return TGKS_EINVAL;
  int r;
  if ((r = ensure_adjoint_buffers(c))) return r;
  const int D = c->g.D;
  // W* of the forward step, unless the caller kept it (P is recomputed
  // too, unused)
  if (!W_star) {
    if ((r = launch_faces(c, W_n, dt_dev, 1, nullptr))) return r;
    if ((r = launch_update(c, 1, W_n, c->Ws, c->P, dt_dev, false))) return r;
  }
  const double* Ws = W_star ? W_star : c->Ws;
  // stage 2 at W*: G* = sum_d (dFA*_d / dW*)^T D_d^T G
  {
    AdjArgs a = adj_args(c, Ws, gW_out, nullptr, 4.0 / 3.0, -8.0 / 3.0, 0.0, 0.0, dt_dev);
    for (int ax = 0; ax < D; ++ax)
      if ((r = reverse_direction(c, a, ax, ax == 0 ? nullptr : c->aWsb, nullptr, c->aWsb))) return r;
  }
  // stage 1 at W^n: G_n = G + G* + sum_d [(dFA_d/dW)^T D^T G* + (dFB_d/dW)^T D^T G]
  {
    AdjArgs a = adj_args(c, W_n, c->aWsb, gW_out, 0.0, 1.0, -1.0 / 3.0, 8.0 / 3.0, dt_dev);
    for (int ax = 0; ax < D; ++ax) {
      if (ax == 0)
        r = reverse_direction(c, a, ax, gW_out, c->aWsb, gW_in);
      else
        r = reverse_direction(c, a, ax, gW_in, nullptr, gW_in);
      if (r) return r;
    }
  }
  return TGKS_OK;
}

}  // extern "C"
