// tgks_opcount.hip -- algorithmic operation counts (tgks_flop_counts): the
// kernels' per-cell and per-face sequences evaluated on the host with the
// operation-counting scalar type.  Host code only, compiled apart from the
// rest of the library (its template instantiations are large).
#include "tgks_internal.hpp"
#include "tgks_opcount.hpp"

using namespace tgks;

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
  const unsigned fl = teno_flag<SEL_EXACT>(Q, c->tn);
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
        teno_gauss(Qw, teno_flag<SEL_EXACT>(Qw, c->tt), v, dv);
        teno_gauss(Qn, teno_flag<SEL_EXACT>(Qn, c->tt), vn, dvn);
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
            teno_gauss(Qw, teno_flag<SEL_EXACT>(Qw, c->tt), v, dv);
            teno_gauss(Qn, teno_flag<SEL_EXACT>(Qn, c->tt), vn, dvn);
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
          teno_gauss(S1w[m1], teno_flag<SEL_EXACT>(S1w[m1], c->tt), v, dv);
          for (int m2 = 0; m2 < 2; ++m2) dv[m2] = dv[m2] * F(1.0 / c->g.dx[2]);
          teno_gauss(S1d[m1], teno_flag<SEL_EXACT>(S1d[m1], c->tt), x, dx_);
          teno_gauss(S1n[m1], teno_flag<SEL_EXACT>(S1n[m1], c->tt), x, dx_);
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
        teno_gauss(Qw, teno_flag<SEL_EXACT>(Qw, c->tt), v, dv);
        teno_gauss(Qn, teno_flag<SEL_EXACT>(Qn, c->tt), vn, dvn);
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

// Comparison schemes (1-D, 2-D): the tangential reconstruction of both
// sides (values and normal slopes), for WENO-Z and TENO5 the face's own
// segment equilibrium (kinetic weighting of its two line-averaged states,
// Eq. 3.12 slopes) and the linear quartic of the five segments at the Gauss
// points (the other four segments are their own faces' work, inputs here),
// and the Gauss-point fluxes.
template <int D, bool NS, int SCHEME>
long long count_face_scheme(const tgks_ctx* c, int stage, tgks_opcount::Tally* detail) {
  constexpr int NC = D + 2;
  constexpr int NG = D == 1 ? 1 : 2;
  constexpr bool SEP = SCHEME >= SCHEME_TENO5;
  tgks_opcount::graph().reset();
  F Wg[2][2][NC], Dg[2][2][D][NC], W0[2][NC], dW0[2][D][NC];
  for (int m = 0; m < NG; ++m)
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < NC; ++q) {
        Wg[m][s][q] = smooth(q < D + 1 ? q : 4, 0.05 * s, 0.1 * m);
        for (int d = 0; d < D; ++d) Dg[m][s][d][q] = F::input(0.01 * (q + 1) * (d + 1));
      }
  if (D == 2) {
    for (int s = 0; s < 2; ++s)
      for (int q = 0; q < NC; ++q) {
        F Qw[5], Qn[5], v[2], dv[2], vn[2], dvn[2];
        for (int r = 0; r < 5; ++r) {
          Qw[r] = smooth(q < 3 ? q : 4, 0.1 * r, 0.0);
          Qn[r] = F::input(0.01 * r);
        }
        scheme_gauss<SCHEME>(Qw, c->sc, v, dv);
        scheme_gauss<SCHEME>(Qn, c->sc, vn, dvn);
        for (int m = 0; m < 2; ++m) {
          Wg[m][s][q] = v[m];
          Dg[m][s][1][q] = dv[m] * F(1.0 / c->g.dx[1]);
          Dg[m][s][0][q] = vn[m];
        }
      }
  }
  if (SEP) {
    // the face's own segment: equilibrium state and its normal slope
    F wl[NC], wr[NC], sl[NC], sr[NC], E[NC], Ex[NC], h0, h1, k0, k1;
    for (int q = 0; q < NC; ++q) {
      wl[q] = smooth(q < D + 1 ? q : 4, 0.0, 0.3);
      wr[q] = smooth(q < D + 1 ? q : 4, 0.05, 0.3);
    }
    Gas<D, F> gl, gr;
    side_w0<D>(wl, c->fc, 1.0, gl, h0, h1, sl);
    side_w0<D>(wr, c->fc, -1.0, gr, k0, k1, sr);
    for (int q = 0; q < NC; ++q) {
      E[q] = sl[q] + sr[q];
      Ex[q] = eq_slope(F::input(1.0 + q), F::input(1.1 + q), F::input(1.2 + q), F::input(1.25 + q)) *
              F(1.0 / c->g.dx[0]);
    }
    for (int q = 0; q < NC; ++q) {
      if (D == 1) {
        W0[0][q] = E[q];
        dW0[0][0][q] = Ex[q];
        continue;
      }
      F Qe[5], Qx[5], v[2], d[2], vx[2], dx_[2];
      for (int r = 0; r < 5; ++r) {
        Qe[r] = r == 2 ? E[q] : F::input(0.9 + 0.01 * r + q);
        Qx[r] = r == 2 ? Ex[q] : F::input(0.1 + 0.01 * r + q);
      }
      SchemeCfg se = c->sc;
      se.q = 6;
      scheme_gauss<SCHEME_TENO5>(Qe, se, v, d);
      scheme_gauss<SCHEME_TENO5>(Qx, se, vx, dx_);
      for (int m = 0; m < 2; ++m) {
        W0[m][q] = v[m];
        dW0[m][D - 1][q] = d[m] * F(1.0 / c->g.dx[1]);
        dW0[m][0][q] = vx[m];
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
    if (SEP)
      gp_flux_eq<D, NS>(Wg[m][0], Wg[m][1], Dg[m][0], Dg[m][1], D == 1 ? (const F*)nullptr : W0[m], dW0[m], fc, dt,
                        Fdt, Fh);
    else
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

// normal reconstruction of one cell and component by a comparison scheme
template <int SCHEME>
long long count_normal_scheme(const tgks_ctx* c) {
  F Q[5], o[4];
  tgks_opcount::graph().reset();
  for (int r = 0; r < 5; ++r) Q[r] = smooth(0, 0.1 * r, 0.0);
  scheme_face<SCHEME>(Q, c->sc, o);
  const F idn(1.0 / c->g.dx[0]);
  F s1 = o[1] * idn, s3 = o[3] * idn;
  (void)s1;
  (void)s3;
  return tgks_opcount::tally().total();
}

template <int D>
long long count_face_dispatch(const tgks_ctx* c, int stage, tgks_opcount::Tally* t) {
  if constexpr (D <= 2) {
    switch (c->p.scheme) {
      case TGKS_SCHEME_WENO_AO:
        return c->ns ? count_face_scheme<D, true, SCHEME_WENO_AO>(c, stage, t)
                     : count_face_scheme<D, false, SCHEME_WENO_AO>(c, stage, t);
      case TGKS_SCHEME_TENO5:
        return c->ns ? count_face_scheme<D, true, SCHEME_TENO5>(c, stage, t)
                     : count_face_scheme<D, false, SCHEME_TENO5>(c, stage, t);
      case TGKS_SCHEME_WENO_Z:
        return c->ns ? count_face_scheme<D, true, SCHEME_WENO_Z>(c, stage, t)
                     : count_face_scheme<D, false, SCHEME_WENO_Z>(c, stage, t);
      default:
        break;
    }
    if (c->p.recon == TGKS_RECON_CHARACTERISTIC)
      return c->ns ? count_face_char<D, true>(c, stage, t) : count_face_char<D, false>(c, stage, t);
  }
  return c->ns ? count_face<D, true>(c, stage, t) : count_face<D, false>(c, stage, t);
}

}  // namespace

extern "C" {

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
  c.tn = teno_cfg(p->ct1, p->ct2, p->eps, p->q);
  c.tt = teno_cfg(p->ct1_tan, p->ct2_tan, p->eps, p->q);
  c.sc = {p->ct1, p->eps, p->q, p->d_hi, p->d_lo, p->eps_w};
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
  long long nr = p->recon == TGKS_RECON_CHARACTERISTIC ? 0 : count_normal(&c);
  if (p->scheme == TGKS_SCHEME_WENO_AO) nr = count_normal_scheme<SCHEME_WENO_AO>(&c);
  if (p->scheme == TGKS_SCHEME_TENO5) nr = count_normal_scheme<SCHEME_TENO5>(&c);
  if (p->scheme == TGKS_SCHEME_WENO_Z) nr = count_normal_scheme<SCHEME_WENO_Z>(&c);
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
