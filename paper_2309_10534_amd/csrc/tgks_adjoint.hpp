// tgks_adjoint.hpp -- reverse mode (vector-Jacobian products) of the
// Gauss-point flux of tgks_device.hpp, written by hand.
//
// The reverse of every forward routine takes the cotangents of its outputs and
// accumulates (+=) the cotangents of its inputs.  Forward intermediates are
// recomputed, not stored.  The time step is a constant and the collision time
// is differentiated through the reconstructed pressures (and, in the viscous
// mode, the equilibrium pressure); a branch (tau == 0, the sign of a pressure
// jump, +1 for equal pressures) keeps the forward's choice.
#pragma once
#include "tgks_device.hpp"

namespace tgks {

template <int D, class R>
struct GasBar {
  R rho, irho, U[D], lam, h;
};

template <int D, class R>
TGKS_HD void zero(GasBar<D, R>& b) {
  b.rho = b.irho = b.lam = b.h = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) b.U[d] = R(0.0);
}

// make_gas: (rho, irho, U, lam, h) of W
template <int D, class R>
TGKS_HD void make_gas_bar(const R* W, double N, const Gas<D, R>& g, const GasBar<D, R>& gb, R* Wb) {
  R ru2 = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) ru2 += g.U[d] * W[d + 1];
  const R eint = W[D + 1] - 0.5 * ru2;
  const R hb = gb.h - gb.lam * (2.0 * (g.lam * g.lam));  // lam = 1/(2h)
  const R eb = hb * ((2.0 / N) * g.irho);
  R irb = gb.irho + hb * ((2.0 / N) * eint);
  Wb[D + 1] += eb;
  const R ru2b = -0.5 * eb;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const R ub = gb.U[d] + ru2b * W[d + 1];
    Wb[d + 1] += ru2b * g.U[d] + ub * g.irho;
    irb += ub * W[d + 1];
  }
  Wb[0] += gb.rho - irb * (g.irho * g.irho);
}

// half_seed: with z = m1 - U m0 (the exp term),
//   dm0/dU = 2 lam z, dm0/dlam = U z, dm1/dU = m0, dm1/dlam = -h z
template <class R>
TGKS_HD void half_seed_bar(R U, R lam, R h, R m0, R m1, R m0b, R m1b, R& Ub, R& lamb) {
  const R z = m1 - U * m0;
  Ub += m0b * (2.0 * lam * z) + m1b * m0;
  lamb += m0b * (U * z) - m1b * (h * z);
}

// table recursion m[k+1] = U m[k] + k h m[k-1], k = 1 .. n-2; mb is consumed
template <class R>
TGKS_HD void table_bar(R U, R h, const R* m, R* mb, int n, R& Ub, R& hb) {
  for (int k = n - 2; k >= 1; --k) {
    const R g = mb[k + 1];
    mb[k] += g * U;
    mb[k - 1] += g * ((double)k * h);
    Ub += g * m[k];
    hb += g * ((double)k * m[k - 1]);
  }
}

template <int D, class R>
struct MomSetBar {
  R m1[NM1];
  R mt[D > 1 ? D - 1 : 1][NMT];
  R xi1, xi2;
};

template <int D, class R>
TGKS_HD void zero(MomSetBar<D, R>& b) {
#pragma unroll
  for (int i = 0; i < NM1; ++i) b.m1[i] = R(0.0);
#pragma unroll
  for (int d = 0; d < (D > 1 ? D - 1 : 1); ++d)
#pragma unroll
    for (int i = 0; i < NMT; ++i) b.mt[d][i] = R(0.0);
  b.xi1 = b.xi2 = R(0.0);
}

template <int D, class R>
TGKS_HD void mono_bar(const MomSet<D, R>& S, MomSetBar<D, R>& Sb, int i, int j, int k, R vb) {
  if (D == 1) {
    Sb.m1[i] += vb;
  } else if (D == 2) {
    Sb.m1[i] += vb * S.mt[0][j];
    Sb.mt[0][j] += vb * S.m1[i];
  } else {
    constexpr int T2 = D >= 3 ? 1 : 0;
    Sb.m1[i] += vb * (S.mt[0][j] * S.mt[T2][k]);
    Sb.mt[0][j] += vb * (S.m1[i] * S.mt[T2][k]);
    Sb.mt[T2][k] += vb * (S.m1[i] * S.mt[0][j]);
  }
}

// gpsi
template <int D, class R>
TGKS_HD void gpsi_bar(const MomSet<D, R>& S, MomSetBar<D, R>& Sb, int i, int j, int k, int l, const R* gb) {
  const R base = mono(S, i, j, k);
  if (l == 0) {
    mono_bar(S, Sb, i, j, k, gb[0] + (0.5 * gb[D + 1]) * S.xi1);
    Sb.xi1 += (0.5 * gb[D + 1]) * base;
    mono_bar(S, Sb, i + 1, j, k, gb[1]);
    if (D >= 2) mono_bar(S, Sb, i, j + 1, k, gb[2]);
    if (D >= 3) mono_bar(S, Sb, i, j, k + 1, gb[D >= 3 ? 3 : 0]);
    const R eb = 0.5 * gb[D + 1];
    mono_bar(S, Sb, i + 2, j, k, eb);
    if (D >= 2) mono_bar(S, Sb, i, j + 2, k, eb);
    if (D >= 3) mono_bar(S, Sb, i, j, k + 2, eb);
  } else {
    const R x = S.xi1;
    mono_bar(S, Sb, i, j, k, gb[0] * x + (0.5 * gb[D + 1]) * S.xi2);
    Sb.xi1 += gb[0] * base;
    Sb.xi2 += (0.5 * gb[D + 1]) * base;
    mono_bar(S, Sb, i + 1, j, k, gb[1] * x);
    Sb.xi1 += gb[1] * mono(S, i + 1, j, k);
    if (D >= 2) {
      mono_bar(S, Sb, i, j + 1, k, gb[2] * x);
      Sb.xi1 += gb[2] * mono(S, i, j + 1, k);
    }
    if (D >= 3) {
      mono_bar(S, Sb, i, j, k + 1, gb[D >= 3 ? 3 : 0] * x);
      Sb.xi1 += gb[D >= 3 ? 3 : 0] * mono(S, i, j, k + 1);
    }
    R e = mono(S, i + 2, j, k);
    if (D >= 2) e = e + mono(S, i, j + 2, k);
    if (D >= 3) e = e + mono(S, i, j, k + 2);
    Sb.xi1 += (0.5 * gb[D + 1]) * e;
    const R eb = (0.5 * gb[D + 1]) * x;
    mono_bar(S, Sb, i + 2, j, k, eb);
    if (D >= 2) mono_bar(S, Sb, i, j + 2, k, eb);
    if (D >= 3) mono_bar(S, Sb, i, j, k + 2, eb);
  }
}

// mpsia: out = s <psi a(psi) u1^i u2^j u3^k>.  ab += cotangent of a; returns
// the cotangent of s.
template <int D, class R>
TGKS_HD R mpsia_bar(const MomSet<D, R>& S, MomSetBar<D, R>& Sb, const R* a, int i, int j, int k, R s, const R* outb,
                    R* ab) {
  constexpr int NC = D + 2;
  R g[NC], t[NC], w[NC];
  R sb = R(0.0);
  // linear terms a_r <psi u_r u1^i u2^j u3^k>
#pragma unroll
  for (int r = 0; r < D + 1; ++r) {
    int ii = i, jj = j, kk = k;
    if (r == 1) ii += 1;
    if (r == 2) jj += 1;
    if (r == 3) kk += 1;
    gpsi<D>(S, ii, jj, kk, 0, g);
    R dot = R(0.0);
    const R as = a[r] * s;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      dot += outb[q] * g[q];
      w[q] = as * outb[q];
    }
    ab[r] += s * dot;
    sb += a[r] * dot;
    gpsi_bar<D>(S, Sb, ii, jj, kk, 0, w);
  }
  // energy term (a_E / 2)(<|u|^2 psi ...> + <xi^2 psi ...>)
  gpsi<D>(S, i + 2, j, k, 0, t);
  if (D >= 2) {
    gpsi<D>(S, i, j + 2, k, 0, g);
#pragma unroll
    for (int q = 0; q < NC; ++q) t[q] += g[q];
  }
  if (D >= 3) {
    gpsi<D>(S, i, j, k + 2, 0, g);
#pragma unroll
    for (int q = 0; q < NC; ++q) t[q] += g[q];
  }
  gpsi<D>(S, i, j, k, 1, g);
  const R ae = 0.5 * a[NC - 1];
  R dot = R(0.0);
  const R as = ae * s;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    dot += outb[q] * (t[q] + g[q]);
    w[q] = as * outb[q];
  }
  ab[NC - 1] += (0.5 * s) * dot;
  sb += ae * dot;
  gpsi_bar<D>(S, Sb, i + 2, j, k, 0, w);
  if (D >= 2) gpsi_bar<D>(S, Sb, i, j + 2, k, 0, w);
  if (D >= 3) gpsi_bar<D>(S, Sb, i, j, k + 2, 0, w);
  gpsi_bar<D>(S, Sb, i, j, k, 1, w);
  return sb;
}

// micro_solve: a = M(U, lam)^-1 b
template <int D, class R>
TGKS_HD void micro_solve_bar(const Gas<D, R>& g, double N, const R* b, const R* a, const R* ab, R* bb,
                             GasBar<D, R>& gb) {
  R ub = R(0.0), u2 = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ub += g.U[d] * b[d + 1];
    u2 += g.U[d] * g.U[d];
  }
  const R lam = g.lam;
  const R aE = a[D + 1];
  const R Q = (2.0 * b[D + 1] - 2.0 * ub) + (u2 - N * g.h) * b[0];
  R aEb = ab[D + 1];
  const R a0b = ab[0];
  bb[0] += a0b;
  const R uab = -a0b;
  aEb += a0b * (-0.5 * (u2 + N * g.h));
  R u2b = a0b * (-0.5 * aE);
  gb.h += a0b * ((-0.5 * N) * aE);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    gb.U[d] += uab * a[d + 1];
    const R adb = ab[d + 1] + uab * g.U[d];
    gb.lam += adb * (2.0 * (b[d + 1] - g.U[d] * b[0]));
    bb[d + 1] += adb * (2.0 * lam);
    bb[0] -= adb * ((2.0 * lam) * g.U[d]);
    gb.U[d] -= adb * ((2.0 * lam) * b[0] + aE);
    aEb -= adb * g.U[d];
  }
  gb.lam += aEb * ((8.0 / N) * lam * Q);
  const R Qb = aEb * ((4.0 / N) * (lam * lam));
  bb[D + 1] += 2.0 * Qb;
  const R ubb = -2.0 * Qb;
  u2b += Qb * b[0];
  gb.h -= Qb * (N * b[0]);
  bb[0] += Qb * (u2 - N * g.h);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    gb.U[d] += ubb * b[d + 1] + 2.0 * u2b * g.U[d];
    bb[d + 1] += ubb * g.U[d];
  }
}

template <int D, class R>
TGKS_HD void zero(Prim<D, R>& p) {
#pragma unroll
  for (int d = 0; d < D; ++d) p.dU[d] = R(0.0);
  p.dp = p.dh = R(0.0);
}

// prim_dir: (dU, dp, dh) along dW
template <int D, class R>
TGKS_HD void prim_dir_bar(const Gas<D, R>& g, double N, const R* dW, const Prim<D, R>& pd, const Prim<D, R>& pb,
                          R* dWb, GasBar<D, R>& gb) {
  R u2 = R(0.0);
#pragma unroll
  for (int e = 0; e < D; ++e) u2 += g.U[e] * g.U[e];
  const R dpb = pb.dp + pb.dh * g.irho;
  gb.h -= pb.dh * (dW[0] * g.irho);
  dWb[0] -= pb.dh * (g.h * g.irho);
  gb.irho += pb.dh * (pd.dp - g.h * dW[0]);
  const R c = (2.0 / N) * dpb;
  dWb[D + 1] += c;
  const R udmb = -c;
  const R u2b = (0.5 * c) * dW[0];
  dWb[0] += (0.5 * c) * u2;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    gb.U[e] += udmb * dW[e + 1] + 2.0 * u2b * g.U[e];
    dWb[e + 1] += udmb * g.U[e];
    const R x = pb.dU[e];
    dWb[e + 1] += x * g.irho;
    dWb[0] -= x * (g.U[e] * g.irho);
    gb.U[e] -= x * (dW[0] * g.irho);
    gb.irho += x * (dW[e + 1] - g.U[e] * dW[0]);
  }
}

// euler_jvp: out = J_k(W) dW
template <int D, class R>
TGKS_HD void euler_jvp_bar(const Gas<D, R>& g, R E, int k, const R* dW, const Prim<D, R>& d, const R* outb, R* dWb,
                           Prim<D, R>& db, GasBar<D, R>& gb, R& Eb) {
  const R p = g.rho * g.h;
  const R mk = g.rho * g.U[k];
  dWb[k + 1] += outb[0];
  R mkb = R(0.0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    const R o = outb[e + 1];
    dWb[k + 1] += o * g.U[e];
    gb.U[e] += o * dW[k + 1];
    mkb += o * d.dU[e];
    db.dU[e] += o * mk;
    if (e == k) db.dp += o;
  }
  const R oE = outb[D + 1];
  db.dU[k] += oE * (E + p);
  Eb += oE * d.dU[k];
  const R pb = oE * d.dU[k];
  gb.U[k] += oE * (dW[D + 1] + d.dp);
  dWb[D + 1] += oE * g.U[k];
  db.dp += oE * g.U[k];
  gb.rho += mkb * g.U[k] + pb * g.h;
  gb.U[k] += mkb * g.rho;
  gb.h += pb * g.rho;
}

// g1d_jvp: out = dG_1d(W) dW
template <int D, class R>
TGKS_HD void g1d_jvp_bar(const Gas<D, R>& g, double N, int d, const R* dW, const Prim<D, R>& q, const R* outb,
                         R* dWb, Prim<D, R>& qb, GasBar<D, R>& gb) {
  const R p = g.rho * g.h;
  const R dp = q.dp;
  R u2 = R(0.0), udu = R(0.0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    u2 += g.U[e] * g.U[e];
    udu += g.U[e] * q.dU[e];
  }
  const R A = g.U[0] * g.U[d];
  const R dA = q.dU[0] * g.U[d] + g.U[0] * q.dU[d];
  const R dr = dW[0];
  const R rdA = dr * A + g.rho * dA;
  const R rA = g.rho * A;
  const R Q = u2 + (N + 4.0) * g.h;
  const R dQ = 2.0 * udu + (N + 4.0) * q.dh;
  R Ub[D];
#pragma unroll
  for (int e = 0; e < D; ++e) Ub[e] = R(0.0);
  R dpb = R(0.0), pb = R(0.0), u2b = R(0.0), udub = R(0.0), hb = R(0.0);
  const R vEb = 0.5 * outb[D + 1];
  R rdAb = vEb * Q;
  const R Qb = vEb * rdA;
  R rAb = vEb * dQ;
  const R dQb = vEb * rA;
  if (d == 0) {
    const R Rr = u2 + (N + 2.0) * g.h;
    const R dRr = 2.0 * udu + (N + 2.0) * q.dh;
    dpb += vEb * Rr;
    pb += vEb * dRr;
    const R Rrb = vEb * dp;
    const R dRrb = vEb * p;
    u2b += Rrb;
    hb += Rrb * (N + 2.0);
    udub += 2.0 * dRrb;
    qb.dh += dRrb * (N + 2.0);
  }
  u2b += Qb;
  hb += Qb * (N + 4.0);
  udub += 2.0 * dQb;
  qb.dh += dQb * (N + 4.0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    const R o = outb[e + 1];
    rdAb += o * g.U[e];
    Ub[e] += o * rdA;
    rAb += o * q.dU[e];
    qb.dU[e] += o * rA;
    if (d == e) {
      dpb += o * g.U[0];
      Ub[0] += o * dp;
      pb += o * q.dU[0];
      qb.dU[0] += o * p;
    }
    if (e == 0) {
      dpb += o * g.U[d];
      Ub[d] += o * dp;
      pb += o * q.dU[d];
      qb.dU[d] += o * p;
    }
    if (d == 0) {
      dpb += o * g.U[e];
      Ub[e] += o * dp;
      pb += o * q.dU[e];
      qb.dU[e] += o * p;
    }
  }
  rdAb += outb[0];
  if (d == 0) dpb += outb[0];
  gb.rho += rAb * A + rdAb * dA + pb * g.h;
  R Ab = rAb * g.rho + rdAb * dr;
  dWb[0] += rdAb * A;
  const R dAb = rdAb * g.rho;
  qb.dU[0] += dAb * g.U[d];
  Ub[d] += dAb * q.dU[0];
  Ub[0] += dAb * q.dU[d];
  qb.dU[d] += dAb * g.U[0];
  Ub[0] += Ab * g.U[d];
  Ub[d] += Ab * g.U[0];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    Ub[e] += udub * q.dU[e] + 2.0 * u2b * g.U[e];
    qb.dU[e] += udub * g.U[e];
    gb.U[e] += Ub[e];
  }
  hb += pb * g.rho;
  gb.h += hb;
  qb.dp += dpb;
}

// heat_combine: y = phi-moment from (f1, f0) about c
template <int D, class R>
TGKS_HD void heat_combine_bar(const R* f1, const R* f0, const R* c, R yb, R* f1b, R* f0b, R* cb) {
  R c2 = R(0.0), s0 = f0[D + 1];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c2 += c[d] * c[d];
    s0 -= c[d] * f0[d + 1];
  }
  s0 += (0.5 * c2) * f0[0];
  const R s1b = yb;
  const R s0b = -yb * c[0];
  cb[0] -= yb * s0;
  f1b[D + 1] += s1b;
  f0b[D + 1] += s0b;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    f1b[d + 1] -= s1b * c[d];
    f0b[d + 1] -= s0b * c[d];
    cb[d] -= s1b * f1[d + 1] + s0b * f0[d + 1];
  }
  const R c2b = 0.5 * (s1b * f1[0] + s0b * f0[0]);
  f1b[0] += (0.5 * c2) * s1b;
  f0b[0] += (0.5 * c2) * s0b;
#pragma unroll
  for (int d = 0; d < D; ++d) cb[d] += 2.0 * c2b * c[d];
}

// the moment tables of one side (as in gp_flux)
template <int D, class R>
TGKS_HD void side_tables(const Gas<D, R>& g, R m0, R m1, double K, MomSet<D, R>& S) {
  half_table(g.U[0], g.h, m0, m1, S.m1);
  tangential_tables<D>(g, S);
  xi_moments<D>(g, K, S);
}

// reverse of side_tables and of the half-space seeds: table cotangents into
// the side's gas cotangents
template <int D, class R>
TGKS_HD void side_tables_bar(const Gas<D, R>& g, R m0, R m1, double K, const MomSet<D, R>& S, MomSetBar<D, R>& Sb,
                             GasBar<D, R>& gb) {
  gb.h += Sb.xi1 * K + Sb.xi2 * ((2.0 * K * (K + 2.0)) * g.h);
#pragma unroll
  for (int d = 1; d < D; ++d) {
    table_bar(g.U[d], g.h, S.mt[d - 1], Sb.mt[d - 1], NMT, gb.U[d], gb.h);
    gb.U[d] += Sb.mt[d - 1][1];
  }
  table_bar(g.U[0], g.h, S.m1, Sb.m1, NM1, gb.U[0], gb.h);
  half_seed_bar(g.U[0], g.lam, g.h, m0, m1, Sb.m1[0], Sb.m1[1], gb.U[0], gb.lam);
}

// Everything one side contributes, recomputed from the side's state and
// slopes: gas state, half-space seeds and moment tables, micro slopes a_d of
// the slopes and A of the time derivative, and Wt = sum_d J_d dW_d.
template <int D, class R>
struct Side {
  Gas<D, R> g;
  R m0, m1;
  MomSet<D, R> S;
  R a[D][D + 2], A[D + 2], Wt[D + 2];
};

// opaque copies of one side's state and slopes (see opaque)
template <int D, class R>
TGKS_HD void opaque_side(const R* W, const R (*dW)[D + 2], R* Wo, R (*dWo)[D + 2]) {
#pragma unroll
  for (int q = 0; q < D + 2; ++q) {
    Wo[q] = opaque(W[q]);
#pragma unroll
    for (int d = 0; d < D; ++d) dWo[d][q] = opaque(dW[d][q]);
  }
}

template <int D, class R>
TGKS_HD void side_forward(const R* Ws, const R (*dW)[D + 2], double sgn, const FluxCfg& P, Side<D, R>& sd) {
  constexpr int NC = D + 2;
  const double N = P.N;
  make_gas<D>(Ws, N, sd.g);
  half_seed(sd.g.U[0], sd.g.lam, sgn, sd.m0, sd.m1);
  side_tables<D>(sd.g, sd.m0, sd.m1, P.K, sd.S);
#pragma unroll
  for (int q = 0; q < NC; ++q) sd.Wt[q] = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    R b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) b[q] = dW[d][q] * sd.g.irho;
    micro_solve<D>(sd.g, N, b, sd.a[d]);
    Prim<D, R> pd;
    prim_dir<D>(sd.g, N, dW[d], pd);
    R jv[NC];
    euler_jvp<D>(sd.g, Ws[D + 1], d, dW[d], pd, jv);
#pragma unroll
    for (int q = 0; q < NC; ++q) sd.Wt[q] += jv[q];
  }
  R b[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) b[q] = -(sd.Wt[q] * sd.g.irho);
  micro_solve<D>(sd.g, N, b, sd.A);
}

// the side's half-space moments of the non-equilibrium part: <u1 psi>,
// sum_d <u1 u_d psi a_d>, <u1 psi A> (and for the heat flux <psi>,
// sum_d <u_d psi a_d>, <psi A>)
template <int D, bool NS, class R>
TGKS_HD void side_moments(const Side<D, R>& sd, R* g1, R* v2, R* v3, R* f0, R* w2, R* w3) {
  constexpr int NC = D + 2;
  gpsi<D>(sd.S, 1, 0, 0, 0, g1);
#pragma unroll
  for (int q = 0; q < NC; ++q) v2[q] = R(0.0);
  if (NS) {
    gpsi<D>(sd.S, 0, 0, 0, 0, f0);
#pragma unroll
    for (int q = 0; q < NC; ++q) w2[q] = R(0.0);
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    int i, j, k;
    unit(d, i, j, k);
    mpsia<D, true>(sd.S, sd.a[d], 1 + i, j, k, R(1.0), v2);
    if (NS) mpsia<D, true>(sd.S, sd.a[d], i, j, k, R(1.0), w2);
  }
  mpsia<D, false>(sd.S, sd.A, 1, 0, 0, R(1.0), v3);
  if (NS) mpsia<D, false>(sd.S, sd.A, 0, 0, 0, R(1.0), w3);
}

// Reverse of gp_flux: given the cotangents Fdtb, Fhb of F(dt), F(dt/2),
// writes the cotangents of Wl, Wr, dWl, dWr (dt is a constant).  The two
// sides' data are recomputed where needed rather than kept, which keeps the
// live state small: forward (sides, then the equilibrium part), reverse of
// the equilibrium part, then one pass per side.
template <int D, bool NS, class R>
TGKS_HD void gp_flux_vjp(const R* Wl, const R* Wr, const R (*dWl)[D + 2], const R (*dWr)[D + 2], const FluxCfg& P,
                         R dt, const R* Fdtb, const R* Fhb, R* Wlb, R* Wrb, R (*dWlb)[D + 2], R (*dWrb)[D + 2]) {
  constexpr int NC = D + 2;
  const double N = P.N;
  // ---- forward: kinetic weighting and the side terms ----
  R W0[NC], dW0[D][NC];
  R Cs[2][3];  // <Fb_id, S_k>, k = S1, S2, S3
  R ps[2];     // side pressures
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    W0[q] = R(0.0);
#pragma unroll
    for (int d = 0; d < D; ++d) dW0[d][q] = R(0.0);
  }
#pragma unroll
  for (int id = 0; id < 2; ++id) Cs[id][0] = Cs[id][1] = Cs[id][2] = R(0.0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    Side<D, R> sd;
    side_forward<D>(s == 0 ? Wl : Wr, s == 0 ? dWl : dWr, s == 0 ? 1.0 : -1.0, P, sd);
    const R rho = sd.g.rho;
    ps[s] = rho * sd.g.h;
    R g[NC];
    gpsi<D>(sd.S, 0, 0, 0, 0, g);
#pragma unroll
    for (int q = 0; q < NC; ++q) W0[q] += rho * g[q];
#pragma unroll
    for (int d = 0; d < D; ++d) mpsia<D, true>(sd.S, sd.a[d], 0, 0, 0, rho, dW0[d]);
    R g1[NC], v2[NC], v3[NC], f0[NC], w2[NC], w3[NC];
    side_moments<D, false>(sd, g1, v2, v3, f0, w2, w3);
#pragma unroll
    for (int id = 0; id < 2; ++id) {
      const R* Fb = id == 0 ? Fdtb : Fhb;
      R c1 = R(0.0), c2 = R(0.0), c3 = R(0.0);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        c1 += Fb[q] * g1[q];
        c2 += Fb[q] * v2[q];
        c3 += Fb[q] * v3[q];
      }
      Cs[id][0] += rho * c1;
      Cs[id][1] += rho * c2;
      Cs[id][2] += rho * c3;
    }
  }
  // ---- forward: equilibrium part ----
  Gas<D, R> g0;
  make_gas<D>(W0, N, g0);
  const R p0 = g0.rho * g0.h;
  const R E0 = W0[D + 1];
  R T1[NC], T2[NC], T3[NC], W0t[NC];
  T1[0] = W0[1];
#pragma unroll
  for (int e = 0; e < D; ++e) T1[e + 1] = W0[1] * g0.U[e] + (e == 0 ? p0 : R(0.0));
  T1[D + 1] = g0.U[0] * (E0 + p0);
#pragma unroll
  for (int q = 0; q < NC; ++q) W0t[q] = T2[q] = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    Prim<D, R> pd;
    prim_dir<D>(g0, N, dW0[d], pd);
    R jv[NC], gv[NC];
    euler_jvp<D>(g0, E0, d, dW0[d], pd, jv);
    g1d_jvp<D>(g0, N, d, dW0[d], pd, gv);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      W0t[q] -= jv[q];
      T2[q] += gv[q];
    }
  }
  {
    Prim<D, R> pt;
    prim_dir<D>(g0, N, W0t, pt);
    euler_jvp<D>(g0, E0, 0, W0t, pt, T3);
  }
  R w2n[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) w2n[q] = -W0t[q];
  R Gq[2] = {R(0.0), R(0.0)}, Hs[3] = {R(0.0), R(0.0), R(0.0)};
  if (NS) {
    Gq[0] = heat_combine<D>(T2, w2n, g0.U);
    Gq[1] = heat_combine<D>(T3, W0t, g0.U);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      R Ws[NC], dW[D][NC];
      opaque_side<D>(s == 0 ? Wl : Wr, s == 0 ? dWl : dWr, Ws, dW);
      Side<D, R> sd;
      side_forward<D>(Ws, dW, s == 0 ? 1.0 : -1.0, P, sd);
      R g1[NC], v2[NC], v3[NC], f0[NC], w2[NC], w3[NC];
      side_moments<D, true>(sd, g1, v2, v3, f0, w2, w3);
      Hs[0] += sd.g.rho * heat_combine<D>(g1, f0, g0.U);
      Hs[1] += sd.g.rho * heat_combine<D>(v2, w2, g0.U);
      Hs[2] += sd.g.rho * heat_combine<D>(v3, w3, g0.U);
    }
  }
  // collision time
  const R S_ = ps[0] + ps[1];
  const R jump = fabs(ps[0] - ps[1]) / S_;
  R tau;
  if (P.tau_mode == 2)
    tau = R(0.0);
  else if (P.tau_mode == 1)
    tau = P.mu / p0 + (P.c2 * jump) * dt;
  else
    tau = (P.c1 + P.c2 * jump) * dt;
  // time coefficients, e^{-dt/tau} = (e^{-dt/(2 tau)})^2
  const R em = tau == 0.0 ? R(0.0) : expm1(-(0.5 * dt) / tau);
  R C[2][6];
  R taub = R(0.0);
  R Gb[2] = {R(0.0), R(0.0)}, Hb[3] = {R(0.0), R(0.0), R(0.0)};
#pragma unroll
  for (int id = 0; id < 2; ++id) {
    const R* Fb = id == 0 ? Fdtb : Fhb;
    const R dl = id == 0 ? dt : 0.5 * dt;
    R e, ome;
    if (tau == 0.0) {
      e = R(0.0);
      ome = R(1.0);
    } else if (id == 1) {
      e = em + 1.0;
      ome = -em;
    } else {
      e = (em + 1.0) * (em + 1.0);
      ome = -em * (em + 2.0);
    }
    const R tt = (tau * tau) * ome;
    C[id][0] = dl - tau * ome;
    C[id][1] = 2.0 * tt - (tau * dl) * (1.0 + e);
    C[id][2] = (0.5 * dl) * dl - tau * dl + tt;
    C[id][3] = tau * ome;
    C[id][4] = (tau * dl) * e - 2.0 * tt;
    C[id][5] = -tt;
    // cotangents of the coefficients: <Fb, X_k>
    R Cb[6];
    Cb[0] = Cb[1] = Cb[2] = R(0.0);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Cb[0] += Fb[q] * T1[q];
      Cb[1] += Fb[q] * T2[q];
      Cb[2] += Fb[q] * T3[q];
    }
    Cb[3] = Cs[id][0];
    Cb[4] = Cs[id][1];
    Cb[5] = Cs[id][2];
    if (NS) {
      const R fe = P.pr_fix * Fb[NC - 1];
      Gb[0] += fe * C[id][1];
      Gb[1] += fe * C[id][2];
      Hb[0] += fe * C[id][3];
      Hb[1] += fe * C[id][4];
      Hb[2] += fe * C[id][5];
      Cb[1] += fe * Gq[0];
      Cb[2] += fe * Gq[1];
      Cb[3] += fe * Hs[0];
      Cb[4] += fe * Hs[1];
      Cb[5] += fe * Hs[2];
    }
    if (tau != 0.0) {
      const R r = dl / tau;
      const R dtt = 2.0 * tau * ome - e * dl;
      const R dC0 = e * r - ome;
      const R dC1 = 2.0 * dtt - dl * (1.0 + e) - (e * dl) * r;
      const R dC2 = dtt - dl;
      const R dC3 = ome - e * r;
      const R dC4 = dl * e + (e * dl) * r - 2.0 * dtt;
      const R dC5 = -dtt;
      taub += ((Cb[0] * dC0 + Cb[1] * dC1) + (Cb[2] * dC2 + Cb[3] * dC3)) + (Cb[4] * dC4 + Cb[5] * dC5);
    }
  }
  // cotangent of X_k: Xb_k = C_k(dt) Fdtb + C_k(dt/2) Fhb
#define XB(k, q) (C[0][k] * Fdtb[q] + C[1][k] * Fhb[q])
  // ---- reverse: collision time ----
  GasBar<D, R> g0b;
  zero(g0b);
  R pb[2] = {R(0.0), R(0.0)};
  if (P.tau_mode != 2 && tau != 0.0) {
    const R jb = taub * (P.c2 * dt);
    if (P.tau_mode == 1) {
      const R p0b = -taub * (P.mu / (p0 * p0));
      g0b.rho += p0b * g0.h;
      g0b.h += p0b * g0.rho;
    }
    // derivative of |x| taken as sign(x), +1 at x = 0 (equal pressures)
    const R sg = ps[0] - ps[1] < 0.0 ? R(-1.0) : R(1.0);
    pb[0] = jb * (sg / S_ - jump / S_);
    pb[1] = jb * (-sg / S_ - jump / S_);
  }
  // ---- reverse: heat moments of the sides (their U0 cotangent only) ----
  if (NS) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      R Ws[NC], dW[D][NC];
      opaque_side<D>(s == 0 ? Wl : Wr, s == 0 ? dWl : dWr, Ws, dW);
      Side<D, R> sd;
      side_forward<D>(Ws, dW, s == 0 ? 1.0 : -1.0, P, sd);
      R g1[NC], v2[NC], v3[NC], f0[NC], w2[NC], w3[NC], t1[NC], t0[NC];
      side_moments<D, true>(sd, g1, v2, v3, f0, w2, w3);
#pragma unroll
      for (int q = 0; q < NC; ++q) t1[q] = t0[q] = R(0.0);
      const R rho = sd.g.rho;
      heat_combine_bar<D>(g1, f0, g0.U, rho * Hb[0], t1, t0, g0b.U);
      heat_combine_bar<D>(v2, w2, g0.U, rho * Hb[1], t1, t0, g0b.U);
      heat_combine_bar<D>(v3, w3, g0.U, rho * Hb[2], t1, t0, g0b.U);
    }
  }
  // ---- reverse: equilibrium part ----
  R T2b[NC], T3b[NC], W0tb[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    T2b[q] = XB(1, q);
    T3b[q] = XB(2, q);
    W0tb[q] = R(0.0);
  }
  if (NS) {
    R w2b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) w2b[q] = R(0.0);
    heat_combine_bar<D>(T2, w2n, g0.U, Gb[0], T2b, w2b, g0b.U);
    heat_combine_bar<D>(T3, W0t, g0.U, Gb[1], T3b, W0tb, g0b.U);
#pragma unroll
    for (int q = 0; q < NC; ++q) W0tb[q] -= w2b[q];
  }
  R E0b = R(0.0);
  {
    Prim<D, R> pt, ptb;
    prim_dir<D>(g0, N, W0t, pt);
    zero(ptb);
    euler_jvp_bar<D>(g0, E0, 0, W0t, pt, T3b, W0tb, ptb, g0b, E0b);
    prim_dir_bar<D>(g0, N, W0t, pt, ptb, W0tb, g0b);
  }
  R dW0b[D][NC];
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int q = 0; q < NC; ++q) dW0b[d][q] = R(0.0);
    Prim<D, R> pd, pdb;
    prim_dir<D>(g0, N, dW0[d], pd);
    zero(pdb);
    R jb[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) jb[q] = -W0tb[q];
    euler_jvp_bar<D>(g0, E0, d, dW0[d], pd, jb, dW0b[d], pdb, g0b, E0b);
    g1d_jvp_bar<D>(g0, N, d, dW0[d], pd, T2b, dW0b[d], pdb, g0b);
    prim_dir_bar<D>(g0, N, dW0[d], pd, pdb, dW0b[d], g0b);
  }
  R W0b[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) W0b[q] = R(0.0);
  {
    // T1 = F_1(W0)
    R T1b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) T1b[q] = XB(0, q);
    const R p0b = T1b[1] + T1b[D + 1] * g0.U[0];
    W0b[1] += T1b[0];
#pragma unroll
    for (int e = 0; e < D; ++e) {
      W0b[1] += T1b[e + 1] * g0.U[e];
      g0b.U[e] += T1b[e + 1] * W0[1];
    }
    g0b.U[0] += T1b[D + 1] * (E0 + p0);
    E0b += T1b[D + 1] * g0.U[0];
    g0b.rho += p0b * g0.h;
    g0b.h += p0b * g0.rho;
  }
  W0b[D + 1] += E0b;
  make_gas_bar<D>(W0, N, g0, g0b, W0b);
  // ---- reverse: one pass per side ----
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    R Ws[NC], dW[D][NC];
    opaque_side<D>(s == 0 ? Wl : Wr, s == 0 ? dWl : dWr, Ws, dW);
    R* Wsb = s == 0 ? Wlb : Wrb;
    R(*dWb)[NC] = s == 0 ? dWlb : dWrb;
    Side<D, R> sd;
    side_forward<D>(Ws, dW, s == 0 ? 1.0 : -1.0, P, sd);
    const Gas<D, R>& g = sd.g;
    const R rho = g.rho;
    GasBar<D, R> gb;
    zero(gb);
    gb.rho += pb[s] * g.h;
    gb.h += pb[s] * rho;
    MomSetBar<D, R> Sb;
    zero(Sb);
    R ab[D][NC], Ab[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Ab[q] = R(0.0);
#pragma unroll
      for (int d = 0; d < D; ++d) ab[d][q] = R(0.0);
    }
    R rb = R(0.0);
    {
      // S1 += rho <u1 psi>, S2 += rho sum_d <u1 u_d psi a_d>, S3 += rho <u1 psi A>
      R g1[NC], ob[NC], xb[NC];
      gpsi<D>(sd.S, 1, 0, 0, 0, g1);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        xb[q] = XB(3, q);
        rb += xb[q] * g1[q];
        ob[q] = rho * xb[q];
      }
      gpsi_bar<D>(sd.S, Sb, 1, 0, 0, 0, ob);
#pragma unroll
      for (int q = 0; q < NC; ++q) xb[q] = XB(4, q);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        int i, j, k;
        unit(d, i, j, k);
        rb += mpsia_bar<D>(sd.S, Sb, sd.a[d], 1 + i, j, k, rho, xb, ab[d]);
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) xb[q] = XB(5, q);
      rb += mpsia_bar<D>(sd.S, Sb, sd.A, 1, 0, 0, rho, xb, Ab);
    }
    if (NS) {
      R g1[NC], v2[NC], v3[NC], f0[NC], w2[NC], w3[NC];
      side_moments<D, true>(sd, g1, v2, v3, f0, w2, w3);
      rb += (Hb[0] * heat_combine<D>(g1, f0, g0.U) + Hb[1] * heat_combine<D>(v2, w2, g0.U)) +
            Hb[2] * heat_combine<D>(v3, w3, g0.U);
      R g1b[NC], f0b[NC], v2b[NC], w2b[NC], v3b[NC], w3b[NC], cdump[D];
#pragma unroll
      for (int q = 0; q < NC; ++q) g1b[q] = f0b[q] = v2b[q] = w2b[q] = v3b[q] = w3b[q] = R(0.0);
#pragma unroll
      for (int d = 0; d < D; ++d) cdump[d] = R(0.0);
      // the U0 cotangents of these terms were taken before the equilibrium
      // reverse; here only the side moments' cotangents
      heat_combine_bar<D>(g1, f0, g0.U, rho * Hb[0], g1b, f0b, cdump);
      heat_combine_bar<D>(v2, w2, g0.U, rho * Hb[1], v2b, w2b, cdump);
      heat_combine_bar<D>(v3, w3, g0.U, rho * Hb[2], v3b, w3b, cdump);
      gpsi_bar<D>(sd.S, Sb, 1, 0, 0, 0, g1b);
      gpsi_bar<D>(sd.S, Sb, 0, 0, 0, 0, f0b);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        int i, j, k;
        unit(d, i, j, k);
        (void)mpsia_bar<D>(sd.S, Sb, sd.a[d], 1 + i, j, k, R(1.0), v2b, ab[d]);
        (void)mpsia_bar<D>(sd.S, Sb, sd.a[d], i, j, k, R(1.0), w2b, ab[d]);
      }
      (void)mpsia_bar<D>(sd.S, Sb, sd.A, 1, 0, 0, R(1.0), v3b, Ab);
      (void)mpsia_bar<D>(sd.S, Sb, sd.A, 0, 0, 0, R(1.0), w3b, Ab);
    }
    {
      // kinetic weighting: W0 += rho <psi>, dW0_d += rho <psi a_d>
      R g[NC], ob[NC];
      gpsi<D>(sd.S, 0, 0, 0, 0, g);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        rb += W0b[q] * g[q];
        ob[q] = rho * W0b[q];
      }
      gpsi_bar<D>(sd.S, Sb, 0, 0, 0, 0, ob);
#pragma unroll
      for (int d = 0; d < D; ++d) rb += mpsia_bar<D>(sd.S, Sb, sd.a[d], 0, 0, 0, rho, dW0b[d], ab[d]);
    }
    gb.rho += rb;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Wsb[q] = R(0.0);
#pragma unroll
      for (int d = 0; d < D; ++d) dWb[d][q] = R(0.0);
    }
    // A = M^-1 (-Wt / rho)
    R b[NC], bb[NC], Wtb[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      b[q] = -(sd.Wt[q] * g.irho);
      bb[q] = R(0.0);
    }
    micro_solve_bar<D>(g, N, b, sd.A, Ab, bb, gb);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Wtb[q] = -(bb[q] * g.irho);
      gb.irho -= bb[q] * sd.Wt[q];
    }
    R Eb = R(0.0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      // Wt += J_d dW_d
      Prim<D, R> pd, pdb;
      prim_dir<D>(g, N, dW[d], pd);
      zero(pdb);
      euler_jvp_bar<D>(g, Ws[D + 1], d, dW[d], pd, Wtb, dWb[d], pdb, gb, Eb);
      prim_dir_bar<D>(g, N, dW[d], pd, pdb, dWb[d], gb);
      // a_d = M^-1 (dW_d / rho)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        b[q] = dW[d][q] * g.irho;
        bb[q] = R(0.0);
      }
      micro_solve_bar<D>(g, N, b, sd.a[d], ab[d], bb, gb);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        dWb[d][q] += bb[q] * g.irho;
        gb.irho += bb[q] * dW[d][q];
      }
    }
    Wsb[D + 1] += Eb;
    side_tables_bar<D>(g, sd.m0, sd.m1, P.K, sd.S, Sb, gb);
    make_gas_bar<D>(Ws, N, g, gb, Wsb);
  }
#undef XB
}

}  // namespace tgks
