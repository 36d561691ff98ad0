// gks_oracle.cpp -- CPU FP64 oracle for the fifth-order TENO-D gas-kinetic
// scheme with the two-stage fourth-order (S2O4) time discretisation of
// Mu, Zhuo, Zhang, Liu & Zhong, "High-order gas-kinetic scheme with TENO class
// reconstruction for the Euler and Navier-Stokes equations" (arXiv:2309.10534).
//
// TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
// reference that the HIP implementation is checked against.  Only the test
// suite, the smoke check and the benchmark's CPU-baseline leg load it; the
// product path never does.  It shares no code, header or table with the HIP
// path.
//
// How it follows the paper:
//  * TENO-D (Sec. 4.2, Eqs. 4.5-4.14): Jiang-Shu smoothness indicators of the
//    three quadratics and of the quartic (Eq. 3.7, the quartic's in Balsara's
//    sum-of-squares form printed for WENO-AO in Sec. 3.2), gamma_k =
//    1/(beta_k+eps)^q, first cut-off on all four candidates, second cut-off on
//    the three small ones, equal linear weights d_k = 1/3.  Interface values
//    and slopes use the coefficients printed in Eqs. 3.2, 4.8, 4.9 and
//    3.22-3.24 (mirrored for the x_{i-1/2} side).
//  * Tangential reconstruction (Sec. 3.2 Steps 1-3, reused for TENO-D at the
//    end of Sec. 4.2): the same selection applied to face-averaged data along
//    the face, the selected polynomial evaluated at the two Gauss points
//    +-1/(2 sqrt 3) (two points per face, Sec. 3.1).
//  * GKS flux (Sec. 2.1, Eqs. 2.2-2.9; kinetic weighting Eqs. 3.25-3.26):
//    every moment is computed by expanding the integrand into monomials of
//    (u1,u2,u3,xi^2) and multiplying one-dimensional Maxwellian moment tables;
//    the micro-slope systems <a psi> = dW/rho and <(a.u + A) psi> = 0 are
//    assembled from those moments and solved by Gaussian elimination.
//  * S2O4 (Sec. 2.2, Eqs. 2.10-2.18): F^n and d_tF^n from the time-integrated
//    fluxes over dt and dt/2, the intermediate state W*, the second-stage
//    d_tF*, the combined flux and the final update, in the paper's order.
//  * Collision time and CFL step (Sec. 5 preamble).
//
// Readings where the paper is silent or garbled:
//  * Eq. 2.5 pairs g_r with H(u); the upwind reading g_l H(u), g_r (1-H(u)) is
//    used, consistent with Eq. 2.6.  Eqs. 3.25-3.26 integrate g^r over u<0.
//  * Reconstruction acts component-wise on the conservative variables (an
//    option reconstructs characteristic fields instead, see below).
//  * Cut-off "0 if chi < C_T, 1 otherwise" is evaluated as
//    !(gamma_k < C_T * sum gamma) (no division, ties keep the stencil).
//  * The smoothness quantities and the candidate values are evaluated with a
//    fixed operation order, constant divisors applied as multiplications by
//    their correctly rounded reciprocals, normal slopes scaled by 1/dx, and
//    without floating-point contraction (build with -ffp-contract=off).
//  * Internal degrees of freedom K = 2/(gamma-1) - D (D = 1, 2, 3).
//  * Navier-Stokes: constant mu; the energy flux is corrected by
//    (1/Pr - 1) * q with q the time-integrated heat flux of f about U0.
//  * A reconstructed or equilibrium state with rho <= 0, p <= 0 or a
//    non-finite value at a Gauss point is counted as a failure.
//  * The no-slip adiabatic wall of the viscous shock tube (Sec. 5.8): ghost
//    cells mirror the interior with every momentum component negated (zero
//    velocity and zero normal temperature gradient at the wall), and the
//    mass and energy fluxes through the wall faces are zero (impermeable;
//    at rest it does no work, adiabatic it conducts no heat); the momentum
//    flux is the flux of the mirrored states.  The symmetry condition there
//    is the reflective kind.
//  * Prescribed (Dirichlet) sides, for the inflow, the post-shock part of
//    the bottom and the moving-shock top of the double Mach reflection
//    (Sec. 5.7), 1-D and 2-D grids: a ghost cell holds the point value of a
//    given state at its centre.  With s the centre's coordinate along the
//    other axis (0 on a 1-D grid), r its coordinate along the side's own
//    axis (both from the domain origin, so r < 0 below a low side) and t the
//    time, it holds state A where s < (s0 + s_n r) + s_t t, otherwise what
//    the side's far kind gives: state B, or the transmissive or reflective
//    image.  The time of stage 1 is t^n, that of stage 2 t^n + dt/2 (W* is
//    the state at the half step).  A corner ghost cell is decided by the
//    x side first when that side is prescribed and gives a state.
//  * Optional first-order fallback (not in the paper, off by default): a
//    Gauss-point state of one side whose density or pressure is
//    not positive or not finite is replaced by the average of that side's
//    cell at the face, with zero slopes, before the flux is evaluated.  The
//    pressure of the test is (gamma - 1) (E - (0.5 sum_a m_a^2) / rho), the
//    sum taken over the momenta in order.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

// ---------------------------------------------------------------------------
// Scalar types: double, and Dual (value plus one directional derivative).
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
static inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
static inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
static inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
static inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
static inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
static inline Dual expm1(Dual a) { return Dual(std::expm1(a.v), std::exp(a.v) * a.d); }
static inline Dual erfc(Dual a) {
  return Dual(std::erfc(a.v), -2.0 / std::sqrt(M_PI) * std::exp(-a.v * a.v) * a.d);
}
static inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }

static inline double val(double a) { return a; }
static inline double val(Dual a) { return a.v; }
using std::erfc;
using std::exp;
using std::expm1;
using std::fabs;
using std::sqrt;

// ---------------------------------------------------------------------------
// Parameters (mirrored by oracle/oracle.py).
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int ndim;
  int n[3];
  double dx[3];
  int bc_lo[3], bc_hi[3];  // 0 periodic, 1 transmissive, 2 reflective, 3 no-slip adiabatic wall,
                           // 4 prescribed (1-D, 2-D)
  double gamma, mu, prandtl;
  int tau_mode;            // 0 inviscid c1 dt + c2 |dp|/(sum p) dt, 1 viscous mu/p0 + ..., 2 zero
  double c1, c2;
  double ct1, ct2, ct1_tan, ct2_tan;
  double eps;
  int q;
  int recon;               // 0 conservative variables, 1 characteristic variables (1-D, 2-D)
  double bc_state[2][5];   // prescribed states A and B (rho, m_0 .. m_{D-1}, E)
  double bc_line[3][2][3]; // per axis and end: (s0, s_n, s_t) of the line bounding state A
  int bc_far[3][2];        // per axis and end: kind beyond the line (1, 2, or 4 = state B)
  int fallback;            // 1: first-order fallback at non-physical Gauss-point states
  int scheme;              // 0 TENO-D (Sec. 4.2), 1 WENO-AO (Sec. 3.2), 2 TENO5 (Sec. 4.1),
                           // 3 WENO-Z (Sec. 3.1); 1-2-3 on 1-D and 2-D grids
  double d_hi, d_lo;       // WENO-AO linear weights of the large and the central small stencil
  double eps_w;            // epsilon of the WENO-AO and WENO-Z weights (Eq. 3.5)
} orc_params;
}

// ---------------------------------------------------------------------------
// TENO-D selection (Sec. 4.2).  Works on the five values Q_{-2..2}.
// ---------------------------------------------------------------------------
// Jiang-Shu indicators of the quadratics on S0, S1, S2 (Eq. 3.7 with q_k = 2)
// and of the quartic on S3 (Eq. 3.7 with q = 4) in Balsara's form with the
// index garble of the printed derivative formulas corrected.
static void teno_beta(const double Q[5], double beta[4]) {
  const double a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  const double k13 = 13.0 / 12.0;
  double t1, t2;
  t1 = (a - 2.0 * b) + c;
  t2 = (a - 4.0 * b) + 3.0 * c;
  beta[0] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (b - 2.0 * c) + d;
  t2 = b - d;
  beta[1] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (c - 2.0 * d) + e;
  t2 = (3.0 * c - 4.0 * d) + e;
  beta[2] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  // p3_x, p3_xx, p3_xxx, p3_xxxx of Sec. 3.2 (cell units)
  const double P1 = (82.0 * (d - b) - 11.0 * (e - a)) * (1.0 / 120.0);
  const double P2 = ((((40.0 * b - 3.0 * a) - 74.0 * c) + 40.0 * d) - 3.0 * e) * (1.0 / 56.0);
  const double P3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
  const double P4 = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) * (1.0 / 24.0);
  const double s1 = P1 + P3 * (1.0 / 10.0);
  const double s2 = P2 + (123.0 / 455.0) * P4;
  beta[3] = (((s1 * s1) + (13.0 / 3.0) * (s2 * s2)) + (781.0 / 20.0) * (P3 * P3)) +
            (1421461.0 / 2275.0) * (P4 * P4);
}

// Flags: bit0 = delta_{3,1}; when bit0 is 0, bits 1..3 = delta_{0,2..2,2}.
static uint8_t teno_select(const double Q[5], double ct1, double ct2, double eps, int qexp) {
  double beta[4];
  teno_beta(Q, beta);
  double g[4];
  for (int k = 0; k < 4; ++k) {
    // gamma_k = 1/(beta_k + eps)^q  (Eq. 4.5), the power by repeated products
    const double bb = beta[k] + eps;
    double pw = 1.0;
    if (qexp == 7) {
      const double b2 = bb * bb;
      const double b4 = b2 * b2;
      pw = (b4 * b2) * bb;
    } else {
      for (int r = 0; r < qexp; ++r) pw = pw * bb;
    }
    g[k] = 1.0 / pw;
  }
  // first cut-off over the four candidates (Eqs. 4.6-4.7)
  const double s4 = ((g[0] + g[1]) + g[2]) + g[3];
  if (!(g[3] < ct1 * s4)) return 1;
  // second cut-off over the small stencils (Eqs. 4.11-4.12)
  const double s3 = (g[0] + g[1]) + g[2];
  uint8_t f = 0;
  for (int k = 0; k < 3; ++k)
    if (!(g[k] < ct2 * s3)) f |= (uint8_t)(2u << k);
  return f;
}

// Interface values and slopes of the selected reconstruction, in cell units:
// out = {value at -1/2, slope at -1/2, value at +1/2, slope at +1/2}.
template <class T>
static void teno_face_values(const T Q[5], uint8_t flag, T out[4]) {
  const T a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  if (flag & 1) {
    // large stencil: Eq. 4.8 / 4.9 and the mirrored x_{i-1/2} forms (Eq. 3.24)
    out[2] = ((((2.0 * a - 13.0 * b) + 47.0 * c) + 27.0 * d) - 3.0 * e) * (1.0 / 60.0);
    out[3] = (((b - 15.0 * c) + 15.0 * d) - e) * (1.0 / 12.0);
    out[0] = ((((27.0 * b - 3.0 * a) + 47.0 * c) - 13.0 * d) + 2.0 * e) * (1.0 / 60.0);
    out[1] = (((a - 15.0 * b) + 15.0 * c) - d) * (1.0 / 12.0);
    return;
  }
  // small stencils (Eqs. 3.2, 3.22-3.23) combined with omega_k = d_k delta_k /
  // sum d_k delta_k, d_k = 1/3 (Eqs. 4.13-4.14)
  T vp[3], dp[3], vm[3], dm[3];
  vp[0] = ((2.0 * a - 7.0 * b) + 11.0 * c) * (1.0 / 6.0);
  vp[1] = ((5.0 * c - b) + 2.0 * d) * (1.0 / 6.0);
  vp[2] = ((2.0 * c + 5.0 * d) - e) * (1.0 / 6.0);
  dp[0] = (a - 3.0 * b) + 2.0 * c;
  dp[1] = d - c;
  dp[2] = d - c;
  vm[0] = ((5.0 * b - a) + 2.0 * c) * (1.0 / 6.0);
  vm[1] = ((2.0 * b + 5.0 * c) - d) * (1.0 / 6.0);
  vm[2] = ((11.0 * c - 7.0 * d) + 2.0 * e) * (1.0 / 6.0);
  dm[0] = c - b;
  dm[1] = c - b;
  dm[2] = (3.0 * d - 2.0 * c) - e;
  double w[3], ws = 0.0;
  for (int k = 0; k < 3; ++k) {
    w[k] = ((flag >> (k + 1)) & 1) ? 1.0 / 3.0 : 0.0;
    ws += w[k];
  }
  for (int k = 0; k < 4; ++k) out[k] = T(0.0);
  for (int k = 0; k < 3; ++k) {
    const double om = w[k] / ws;
    out[0] += om * vm[k];
    out[1] += om * dm[k];
    out[2] += om * vp[k];
    out[3] += om * dp[k];
  }
}

// Monomial coefficients (cell units, x in [-1/2, 1/2]) of the cell-average
// matching polynomials p_k (Sec. 3.1) and p_3 (Sec. 3.2).
template <class T>
static void teno_poly(const T Q[5], int k, T co[5]) {
  const T a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  for (int i = 0; i < 5; ++i) co[i] = T(0.0);
  switch (k) {
    case 0:
      co[0] = ((23.0 * c + 2.0 * b) - a) / 24.0;
      co[1] = ((3.0 * c - 4.0 * b) + a) / 2.0;
      co[2] = ((c - 2.0 * b) + a) / 2.0;
      break;
    case 1:
      co[0] = ((26.0 * c - d) - b) / 24.0;
      co[1] = (d - b) / 2.0;
      co[2] = ((d + b) - 2.0 * c) / 2.0;
      break;
    case 2:
      co[0] = ((23.0 * c + 2.0 * d) - e) / 24.0;
      co[1] = ((4.0 * d - 3.0 * c) - e) / 2.0;
      co[2] = ((c - 2.0 * d) + e) / 2.0;
      break;
    default:
      co[0] = ((2134.0 * c - 116.0 * (d + b)) + 9.0 * (e + a)) / 1920.0;
      co[1] = (34.0 * (d - b) - 5.0 * (e - a)) / 48.0;
      co[2] = ((12.0 * (d + b) - 22.0 * c) - (e + a)) / 16.0;
      co[3] = ((e - a) - 2.0 * (d - b)) / 12.0;
      co[4] = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) / 24.0;
  }
}

// Selected polynomial evaluated at the two Gauss points s = -+1/(2 sqrt 3):
// out = {value at s-, slope at s-, value at s+, slope at s+} (cell units).
template <class T>
static void teno_gauss_values(const T Q[5], uint8_t flag, T out[4]) {
  const double sg[2] = {-0.5 / std::sqrt(3.0), 0.5 / std::sqrt(3.0)};
  for (int k = 0; k < 4; ++k) out[k] = T(0.0);
  double w[4] = {0, 0, 0, 0};
  if (flag & 1) {
    w[3] = 1.0;
  } else {
    double ws = 0.0;
    for (int k = 0; k < 3; ++k) {
      w[k] = ((flag >> (k + 1)) & 1) ? 1.0 / 3.0 : 0.0;
      ws += w[k];
    }
    for (int k = 0; k < 3; ++k) w[k] /= ws;
  }
  for (int k = 0; k < 4; ++k) {
    if (w[k] == 0.0) continue;
    T co[5];
    teno_poly(Q, k, co);
    for (int m = 0; m < 2; ++m) {
      const double s = sg[m];
      T v = co[4];
      for (int i = 3; i >= 0; --i) v = v * s + co[i];
      T dv = 4.0 * co[4];
      for (int i = 3; i >= 1; --i) dv = dv * s + double(i) * co[i];
      out[2 * m] += w[k] * v;
      out[2 * m + 1] += w[k] * dv;
    }
  }
}

// The same values and slopes in one fixed evaluation order (monomial
// coefficients as multiples of correctly rounded reciprocals, even and odd
// parts in the Gauss-point coordinate), for the 3-D first sweep, whose
// results are the inputs of the second sweep's selections: identical data
// must give identical selections in every implementation (reading R8).
template <class T>
static void teno_gauss_canonical(const T Q[5], uint8_t flag, T out[4]) {
  const T a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  const double s = 0.28867513459481288225;  // 1/(2 sqrt 3)
  T c0, c1, c2, c3 = T(0.0), c4 = T(0.0);
  if (flag & 1) {
    c0 = ((2134.0 * c - 116.0 * (d + b)) + 9.0 * (e + a)) * (1.0 / 1920.0);
    c1 = (34.0 * (d - b) - 5.0 * (e - a)) * (1.0 / 48.0);
    c2 = ((12.0 * (d + b) - 22.0 * c) - (e + a)) * (1.0 / 16.0);
    c3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
    c4 = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) * (1.0 / 24.0);
  } else {
    // equal weights of the surviving quadratics (1, 1/2 or 1/3 each)
    const int cnt = ((flag >> 1) & 1) + ((flag >> 2) & 1) + ((flag >> 3) & 1);
    const double inv = cnt == 1 ? 1.0 : (cnt == 2 ? 0.5 : 1.0 / 3.0);
    T s0 = T(0.0), s1 = T(0.0), s2 = T(0.0);
    if (flag & 2) {
      s0 = s0 + ((23.0 * c + 2.0 * b) - a) * (1.0 / 24.0);
      s1 = s1 + ((3.0 * c - 4.0 * b) + a) * 0.5;
      s2 = s2 + ((c - 2.0 * b) + a) * 0.5;
    }
    if (flag & 4) {
      s0 = s0 + ((26.0 * c - d) - b) * (1.0 / 24.0);
      s1 = s1 + (d - b) * 0.5;
      s2 = s2 + ((d + b) - 2.0 * c) * 0.5;
    }
    if (flag & 8) {
      s0 = s0 + ((23.0 * c + 2.0 * d) - e) * (1.0 / 24.0);
      s1 = s1 + ((4.0 * d - 3.0 * c) - e) * 0.5;
      s2 = s2 + ((c - 2.0 * d) + e) * 0.5;
    }
    c0 = s0 * inv;
    c1 = s1 * inv;
    c2 = s2 * inv;
  }
  const double ss = s * s;
  const T even = c0 + ss * (c2 + ss * c4);
  const T odd = s * (c1 + ss * c3);
  const T deven = c1 + (3.0 * ss) * c3;
  const T dodd = s * (2.0 * c2 + (4.0 * ss) * c4);
  out[0] = even - odd;
  out[1] = deven - dodd;
  out[2] = even + odd;
  out[3] = deven + dodd;
}

template <class T>
static uint8_t select_T(const T Q[5], double ct1, double ct2, double eps, int q) {
  double qv[5];
  for (int i = 0; i < 5; ++i) qv[i] = val(Q[i]);
  return teno_select(qv, ct1, ct2, eps, q);
}

// ---------------------------------------------------------------------------
// The comparison schemes of the paper, each on the same five values Q_{-2..2}
// and the same candidate polynomials p_0..p_2 (Sec. 3.1) and p_3 (Sec. 3.2).
//  * WENO-AO (Sec. 3.2): linear weights d_3 = d_Hi, d_0 = d_2 =
//    (1 - d_Hi)(1 - d_Lo)/2, d_1 = (1 - d_Hi) d_Lo; WENO-Z type weights
//    omega_k = d_k (1 + (tau / (beta_k + eps))^2) (Eq. 3.5 with the ratio
//    squared, as Table 2 requires) with
//    tau = (|b3 - b0| + |b3 - b1| + |b3 - b2|) / 3, normalised over k = 0..3;
//    p_AO = w3 (p_3 / d_3 - sum_k d_k / d_3 p_k) + sum_k w_k p_k, evaluated
//    (value and derivative) wherever a value or slope is needed: the
//    interfaces (Eqs. 3.22-3.24 are its pieces) and the Gauss points.
//  * WENO-Z (Sec. 3.1): small stencils only, omega_k = d_k (1 + tau /
//    (beta_k + eps)), tau = |b0 - b2| (Eqs. 3.5-3.8), d = (0.1, 0.6, 0.3) at
//    x_{i+1/2}, mirrored at x_{i-1/2}, and at a Gauss point the linear
//    weights that reproduce p_3 there.
//  * TENO5 (Sec. 4.1): gamma_k = (C + tau / (beta_k + eps))^q, C = 1,
//    tau = |b0 - b2|, cut-off delta_k = 0 where gamma_k / sum gamma < C_T
//    (evaluated as gamma_k < C_T sum gamma), omega_k = d_k delta_k /
//    sum d_j delta_j (Eqs. 4.1-4.4) with the same linear weights.
//  * WENO-Z and TENO5 give the non-equilibrium interface values only; the
//    slopes come from the quadratic with the cell average and the two
//    interface values (Eq. 3.11).  Along a face (Gauss points) the slope is
//    that quadratic's derivative at the Gauss point, built from the face
//    segment's line average and its two end values.
// ---------------------------------------------------------------------------
static const double GPW = 1.7320508075688772 / 1080.0;  // sqrt(3)/1080

// linear weights of p_0..p_2 that reproduce p_3 at x = -1/2 (where 0),
// +1/2 (1), the Gauss point -1/(2 sqrt 3) (2) or +1/(2 sqrt 3) (3)
static void lin_weights(int where, double d[3]) {
  switch (where) {
    case 0: d[0] = 0.3; d[1] = 0.6; d[2] = 0.1; break;
    case 1: d[0] = 0.1; d[1] = 0.6; d[2] = 0.3; break;
    case 2: d[0] = 7.0 / 36.0 + GPW; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 - GPW; break;
    default: d[0] = 7.0 / 36.0 - GPW; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 + GPW;
  }
}

// TENO5 cut-offs: bit k = delta_k
static uint8_t teno5_select(const double Q[5], double ct, double eps, int qexp) {
  double b[4];
  teno_beta(Q, b);
  const double tau = std::fabs(b[0] - b[2]);
  double g[3];
  for (int k = 0; k < 3; ++k) {
    const double t = 1.0 + tau / (b[k] + eps);
    double pw = 1.0;
    if (qexp == 6) {
      const double t2 = t * t;
      const double t4 = t2 * t2;
      pw = t4 * t2;
    } else {
      for (int r = 0; r < qexp; ++r) pw = pw * t;
    }
    g[k] = pw;
  }
  const double sg = (g[0] + g[1]) + g[2];
  uint8_t f = 0;
  for (int k = 0; k < 3; ++k)
    if (!(g[k] < ct * sg)) f |= (uint8_t)(1u << k);
  return f;
}

// normalised weights of p_0..p_2 at point `where` (WENO-Z or TENO5)
static void small_weights(const orc_params& P, const double Q[5], int where, uint8_t flag, double ob[3]) {
  double d[3];
  lin_weights(where, d);
  if (P.scheme == 2) {
    double S = 0.0;
    for (int k = 0; k < 3; ++k) S = S + ((flag >> k) & 1 ? d[k] : 0.0);
    for (int k = 0; k < 3; ++k) ob[k] = (flag >> k) & 1 ? d[k] / S : 0.0;
    return;
  }
  double b[4];
  teno_beta(Q, b);
  const double tau = std::fabs(b[0] - b[2]);
  double om[3], S = 0.0;
  for (int k = 0; k < 3; ++k) {
    om[k] = d[k] * (1.0 + tau / (b[k] + P.eps_w));
    S = S + om[k];
  }
  for (int k = 0; k < 3; ++k) ob[k] = om[k] / S;
}

// coefficients of p_0..p_3 in the WENO-AO polynomial
static void ao_weights(const orc_params& P, const double Q[5], double w[4]) {
  double b[4];
  teno_beta(Q, b);
  const double dh = P.d_hi, dl = P.d_lo;
  const double d[4] = {(1.0 - dh) * (1.0 - dl) / 2.0, (1.0 - dh) * dl, (1.0 - dh) * (1.0 - dl) / 2.0, dh};
  const double tau = (std::fabs(b[3] - b[0]) + std::fabs(b[3] - b[1]) + std::fabs(b[3] - b[2])) / 3.0;
  double om[4], S = 0.0;
  for (int k = 0; k < 4; ++k) {
    // the ratio enters squared (Table 2: the unsquared form of Eq. 3.5
    // misses the printed errors by 1-4 %, the squared one matches them)
    const double r = tau / (b[k] + P.eps_w);
    om[k] = d[k] * (1.0 + r * r);
    S = S + om[k];
  }
  double ob[4];
  for (int k = 0; k < 4; ++k) ob[k] = om[k] / S;
  w[3] = ob[3] / d[3];
  for (int k = 0; k < 3; ++k) w[k] = ob[k] - ob[3] * d[k] / d[3];
}

// value and derivative (cell units) at x of sum_k w[k] p_k
template <class T>
static void poly_combo(const T Q[5], const double w[4], double x, T& v, T& dv) {
  v = T(0.0);
  dv = T(0.0);
  for (int k = 0; k < 4; ++k) {
    if (w[k] == 0.0) continue;
    T co[5];
    teno_poly(Q, k, co);
    T pv = co[4];
    for (int i = 3; i >= 0; --i) pv = pv * x + co[i];
    T pd = 4.0 * co[4];
    for (int i = 3; i >= 1; --i) pd = pd * x + double(i) * co[i];
    v += w[k] * pv;
    dv += w[k] * pd;
  }
}

// interface values of p_0..p_2: vm at x_{i-1/2}, vp at x_{i+1/2} (Eq. 3.2 and
// its mirror image)
template <class T>
static void small_face_values(const T Q[5], T vm[3], T vp[3]) {
  const T a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  vp[0] = ((2.0 * a - 7.0 * b) + 11.0 * c) * (1.0 / 6.0);
  vp[1] = ((5.0 * c - b) + 2.0 * d) * (1.0 / 6.0);
  vp[2] = ((2.0 * c + 5.0 * d) - e) * (1.0 / 6.0);
  vm[0] = ((5.0 * b - a) + 2.0 * c) * (1.0 / 6.0);
  vm[1] = ((2.0 * b + 5.0 * c) - d) * (1.0 / 6.0);
  vm[2] = ((11.0 * c - 7.0 * d) + 2.0 * e) * (1.0 / 6.0);
}

// WENO-Z / TENO5 interface values v(-1/2), v(+1/2)
template <class T>
static uint8_t zt_face_values(const orc_params& P, const T Q[5], T& vm_out, T& vp_out) {
  double q[5];
  for (int i = 0; i < 5; ++i) q[i] = val(Q[i]);
  const uint8_t f = P.scheme == 2 ? teno5_select(q, P.ct1, P.eps, P.q) : 0;
  double om[3], op[3];
  small_weights(P, q, 0, f, om);
  small_weights(P, q, 1, f, op);
  T vm[3], vp[3];
  small_face_values(Q, vm, vp);
  vm_out = T(0.0);
  vp_out = T(0.0);
  for (int k = 0; k < 3; ++k) {
    vm_out += om[k] * vm[k];
    vp_out += op[k] * vp[k];
  }
  return f;
}

// Normal reconstruction of a comparison scheme: {v(-1/2), s(-1/2), v(+1/2),
// s(+1/2)} in cell units; returns the TENO5 cut-off flags (0 otherwise)
template <class T>
static uint8_t scheme_face(const orc_params& P, const T Q[5], T out[4]) {
  if (P.scheme == 1) {
    double q[5], w[4];
    for (int i = 0; i < 5; ++i) q[i] = val(Q[i]);
    ao_weights(P, q, w);
    poly_combo(Q, w, -0.5, out[0], out[1]);
    poly_combo(Q, w, 0.5, out[2], out[3]);
    return 0;
  }
  T vm, vp;
  const uint8_t f = zt_face_values(P, Q, vm, vp);
  // the quadratic with average Q_0 and end values vm, vp (Eq. 3.11)
  out[0] = vm;
  out[1] = -2.0 * ((2.0 * vm + vp) - 3.0 * Q[2]);
  out[2] = vp;
  out[3] = 2.0 * ((vm + 2.0 * vp) - 3.0 * Q[2]);
  return f;
}

// Tangential reconstruction of a comparison scheme at the two Gauss points:
// {v(s-), d(s-), v(s+), d(s+)} in cell units; returns the TENO5 flags
template <class T>
static uint8_t scheme_gauss(const orc_params& P, const T Q[5], T out[4]) {
  const double sg[2] = {-0.5 / std::sqrt(3.0), 0.5 / std::sqrt(3.0)};
  double q[5];
  for (int i = 0; i < 5; ++i) q[i] = val(Q[i]);
  if (P.scheme == 1) {
    double w[4];
    ao_weights(P, q, w);
    for (int m = 0; m < 2; ++m) poly_combo(Q, w, sg[m], out[2 * m], out[2 * m + 1]);
    return 0;
  }
  T vm, vp;
  const uint8_t f = zt_face_values(P, Q, vm, vp);
  const T c1 = vp - vm, c2 = 3.0 * (vm + vp) - 6.0 * Q[2];
  for (int m = 0; m < 2; ++m) {
    double ob[3], w[4] = {0, 0, 0, 0};
    small_weights(P, q, 2 + m, f, ob);
    for (int k = 0; k < 3; ++k) w[k] = ob[k];
    T dv;
    poly_combo(Q, w, sg[m], out[2 * m], dv);
    out[2 * m + 1] = c1 + (2.0 * sg[m]) * c2;
  }
  return f;
}

// the selection and reconstruction of the configured scheme: normal (face
// values and slopes) or tangential (Gauss points)
template <class T>
static uint8_t recon_face(const orc_params& P, const T Q[5], T out[4]) {
  if (P.scheme != 0) return scheme_face(P, Q, out);
  const uint8_t f = select_T(Q, P.ct1, P.ct2, P.eps, P.q);
  teno_face_values(Q, f, out);
  return f;
}

template <class T>
static uint8_t recon_gauss(const orc_params& P, const T Q[5], T out[4]) {
  if (P.scheme != 0) return scheme_gauss(P, Q, out);
  const uint8_t f = select_T(Q, P.ct1_tan, P.ct2_tan, P.eps, P.q);
  teno_gauss_values(Q, f, out);
  return f;
}

// ---------------------------------------------------------------------------
// Maxwellian moments (Sec. 2.1).  One-dimensional tables of
// <u^n> = int u^n sqrt(lambda/pi) exp(-lambda (u-U)^2) du over the full line
// (kind 0), u > 0 (kind +1) or u < 0 (kind -1), and of the internal variable:
// <xi^(2l)> over K Gaussian degrees of freedom.
// ---------------------------------------------------------------------------
static const int NM = 10;  // table length (powers 0..9)

template <class T>
static void mom1d(T U, T lam, int kind, T m[NM]) {
  if (kind == 0) {
    m[0] = T(1.0);
    m[1] = U;
  } else {
    const double sgn = kind > 0 ? 1.0 : -1.0;
    const T sl = sqrt(lam);
    m[0] = 0.5 * erfc(-sgn * (sl * U));
    m[1] = U * m[0] + sgn * 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
  }
  for (int n = 1; n + 1 < NM; ++n) m[n + 1] = U * m[n] + (double(n) / 2.0) * m[n - 1] / lam;
}

template <class T>
static void momxi(double K, T lam, T m[4]) {
  m[0] = T(1.0);
  for (int l = 1; l < 4; ++l) m[l] = m[l - 1] * (K + 2.0 * (l - 1)) / (2.0 * lam);
}

// A polynomial in (u1, u2, u3, xi^2) as a list of monomials.
template <class T>
struct Poly {
  struct Term {
    int e[4];
    T c;
  };
  std::vector<Term> t;
  void add(int e0, int e1, int e2, int e3, T c) {
    for (auto& x : t)
      if (x.e[0] == e0 && x.e[1] == e1 && x.e[2] == e2 && x.e[3] == e3) {
        x.c += c;
        return;
      }
    Term n;
    n.e[0] = e0; n.e[1] = e1; n.e[2] = e2; n.e[3] = e3; n.c = c;
    t.push_back(n);
  }
  void add(const Poly& o, T s) {
    for (auto& x : o.t) add(x.e[0], x.e[1], x.e[2], x.e[3], s * x.c);
  }
};

template <class T>
static Poly<T> mul(const Poly<T>& A, const Poly<T>& B) {
  Poly<T> r;
  for (auto& x : A.t)
    for (auto& y : B.t)
      r.add(x.e[0] + y.e[0], x.e[1] + y.e[1], x.e[2] + y.e[2], x.e[3] + y.e[3], x.c * y.c);
  return r;
}

// psi_alpha in the face frame: 1, u_1..u_D, (|u|^2 + xi^2)/2  (Eq. 2.3).
template <class T>
static Poly<T> psi(int D, int alpha) {
  Poly<T> p;
  if (alpha == 0) {
    p.add(0, 0, 0, 0, T(1.0));
  } else if (alpha <= D) {
    int e[3] = {0, 0, 0};
    e[alpha - 1] = 1;
    p.add(e[0], e[1], e[2], 0, T(1.0));
  } else {
    for (int d = 0; d < D; ++d) {
      int e[3] = {0, 0, 0};
      e[d] = 2;
      p.add(e[0], e[1], e[2], 0, T(0.5));
    }
    p.add(0, 0, 0, 1, T(0.5));
  }
  return p;
}

// u_d as a polynomial
template <class T>
static Poly<T> uvar(int d) {
  Poly<T> p;
  int e[3] = {0, 0, 0};
  e[d] = 1;
  p.add(e[0], e[1], e[2], 0, T(1.0));
  return p;
}

// sum_beta a_beta psi_beta
template <class T>
static Poly<T> micro(int D, const T* a) {
  Poly<T> p;
  for (int b = 0; b < D + 2; ++b) p.add(psi<T>(D, b), a[b]);
  return p;
}

// A Maxwellian state with its moment tables; the normal (u1) table may be a
// half-space table.
template <class T>
struct Maxw {
  int D;
  T rho, lam;
  T U[3];
  T m[3][NM];
  T mx[4];
  void build(int D_, double K, const T* W, int kind) {
    D = D_;
    rho = W[0];
    T ke = T(0.0);
    for (int d = 0; d < 3; ++d) U[d] = T(0.0);
    for (int d = 0; d < D; ++d) {
      U[d] = W[1 + d] / rho;
      ke += U[d] * U[d];
    }
    // rho E = rho |U|^2 / 2 + (K + D) rho / (4 lambda)
    lam = (K + D) * rho / (4.0 * (W[D + 1] - 0.5 * rho * ke));
    for (int d = 0; d < 3; ++d) mom1d(U[d], lam, d == 0 ? kind : 0, m[d]);
    momxi(K, lam, mx);
  }
  T mono(const int e[4]) const { return ((m[0][e[0]] * m[1][e[1]]) * m[2][e[2]]) * mx[e[3]]; }
  // moment of a polynomial per unit density
  T mom(const Poly<T>& P) const {
    T s = T(0.0);
    for (auto& x : P.t) s += x.c * mono(x.e);
    return s;
  }
  T pressure() const { return rho / (2.0 * lam); }
};

// Solve M x = b (n <= 5) by Gaussian elimination with partial pivoting.
template <class T>
static void gauss_solve(int n, T M[5][5], T b[5], T x[5]) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(val(M[i][k])) > std::fabs(val(M[piv][k]))) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(M[k][j], M[piv][j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const T f = M[i][k] / M[k][k];
      for (int j = k; j < n; ++j) M[i][j] -= f * M[k][j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = b[i];
    for (int j = i + 1; j < n; ++j) s -= M[i][j] * x[j];
    x[i] = s / M[i][i];
  }
}

// Micro coefficients a with <a psi> = rhs over the full Maxwellian g (Eq. 2.7).
template <class T>
static void solve_micro(const Maxw<T>& full, const T* rhs, T* a) {
  const int D = full.D, nc = D + 2;
  T M[5][5], b[5], x[5];
  for (int i = 0; i < nc; ++i) {
    const Poly<T> pi = psi<T>(D, i);
    for (int j = 0; j < nc; ++j) M[i][j] = full.mom(mul(pi, psi<T>(D, j)));
    b[i] = rhs[i];
  }
  gauss_solve(nc, M, b, x);
  for (int i = 0; i < nc; ++i) a[i] = x[i];
}

static inline bool state_ok(double rho, double p) {
  return rho > 0.0 && p > 0.0 && std::isfinite(rho) && std::isfinite(p);
}

// Time-integrated interface flux at one Gauss point, face frame (u1 normal).
// Wl, Wr: reconstructed states; dWl[d], dWr[d]: their derivatives along frame
// axis d; dt: full step (enters tau); delta: integration interval.
// Outputs F[nc] = F(delta); optionally W0 and dW0 (kinetic weighting).
template <class T>
static int gp_flux(const orc_params& P, int D, const T* Wl, const T* Wr, const T dWl[3][5],
                   const T dWr[3][5], double dt, int ndelta, const double* delta, T F[][5],
                   T* W0out, T dW0out[3][5], const T* W0in = nullptr, const T (*dW0in)[5] = nullptr) {
  const int nc = D + 2;
  const double K = 2.0 / (P.gamma - 1.0) - D;
  int bad = 0;
  Maxw<T> hl, hr, fl, fr, g0;
  hl.build(D, K, Wl, +1);
  hr.build(D, K, Wr, -1);
  fl.build(D, K, Wl, 0);
  fr.build(D, K, Wr, 0);
  if (!state_ok(val(hl.rho), val(hl.pressure())) || !state_ok(val(hr.rho), val(hr.pressure()))) bad = 1;

  Poly<T> ps[5];
  for (int a = 0; a < nc; ++a) ps[a] = psi<T>(D, a);

  // Equilibrium state by kinetic weighting (Eq. 2.6 / 3.25), or given
  // (separately reconstructed, Sec. 3.1)
  T W0[5];
  for (int a = 0; a < nc; ++a) W0[a] = W0in ? W0in[a] : hl.rho * hl.mom(ps[a]) + hr.rho * hr.mom(ps[a]);

  // Non-equilibrium micro slopes a^k_d: <a psi> = dW^k_d / rho_k (Eq. 2.7).
  T al[3][5], ar[3][5];
  for (int d = 0; d < D; ++d) {
    T bl[5], br[5];
    for (int a = 0; a < nc; ++a) {
      bl[a] = dWl[d][a] / fl.rho;
      br[a] = dWr[d][a] / fr.rho;
    }
    solve_micro(fl, bl, al[d]);
    solve_micro(fr, br, ar[d]);
  }
  // Equilibrium slopes by kinetic weighting (Eq. 2.6 lines 2-3 / 3.26), or
  // given (Eq. 3.12 and its tangential reconstruction)
  T dW0[3][5];
  for (int d = 0; d < D; ++d) {
    const Poly<T> ml = micro(D, al[d]), mr = micro(D, ar[d]);
    for (int a = 0; a < nc; ++a)
      dW0[d][a] = dW0in ? dW0in[d][a] : hl.rho * hl.mom(mul(ps[a], ml)) + hr.rho * hr.mom(mul(ps[a], mr));
  }
  if (W0out)
    for (int a = 0; a < nc; ++a) W0out[a] = W0[a];
  if (dW0out)
    for (int d = 0; d < D; ++d)
      for (int a = 0; a < nc; ++a) dW0out[d][a] = dW0[d][a];

  g0.build(D, K, W0, 0);
  if (!state_ok(val(g0.rho), val(g0.pressure()))) bad = 1;

  // Equilibrium micro slopes abar_d and time derivative Abar (Eq. 2.7).
  T ab[3][5];
  for (int d = 0; d < D; ++d) {
    T b[5];
    for (int a = 0; a < nc; ++a) b[a] = dW0[d][a] / g0.rho;
    solve_micro(g0, b, ab[d]);
  }
  Poly<T> ua0;  // sum_d u_d abar_d(psi)
  for (int d = 0; d < D; ++d) ua0.add(mul(uvar<T>(d), micro(D, ab[d])), T(1.0));
  T Ab[5];
  {
    T b[5];
    for (int a = 0; a < nc; ++a) b[a] = -g0.mom(mul(ps[a], ua0));
    solve_micro(g0, b, Ab);
  }
  // Non-equilibrium time derivatives A^l, A^r over the full g_l, g_r.
  Poly<T> ual, uar;
  for (int d = 0; d < D; ++d) {
    ual.add(mul(uvar<T>(d), micro(D, al[d])), T(1.0));
    uar.add(mul(uvar<T>(d), micro(D, ar[d])), T(1.0));
  }
  T Al[5], Ar[5];
  {
    T bl[5], br[5];
    for (int a = 0; a < nc; ++a) {
      bl[a] = -fl.mom(mul(ps[a], ual));
      br[a] = -fr.mom(mul(ps[a], uar));
    }
    solve_micro(fl, bl, Al);
    solve_micro(fr, br, Ar);
  }
  const Poly<T> pAb = micro(D, Ab), pAl = micro(D, Al), pAr = micro(D, Ar);

  // Collision time (Sec. 5 preamble).
  const T pl = fl.pressure(), pr = fr.pressure();
  T tau;
  const T jump = fabs(pl - pr) / (pl + pr);
  if (P.tau_mode == 2)
    tau = T(0.0);
  else if (P.tau_mode == 1)
    tau = P.mu / g0.pressure() + P.c2 * jump * dt;
  else
    tau = P.c1 * dt + P.c2 * jump * dt;

  // Flux weights u1 psi_alpha (Eq. 2.9), plus the heat-flux weight for the
  // Prandtl correction: (u1-U0_1)(|u-U0|^2 + xi^2)/2.
  Poly<T> w[6];
  const Poly<T> u1 = uvar<T>(0);
  for (int a = 0; a < nc; ++a) w[a] = mul(u1, ps[a]);
  const bool ns = P.mu > 0.0 && P.prandtl != 1.0;
  if (ns) {
    Poly<T> c1p;
    c1p.add(1, 0, 0, 0, T(1.0));
    c1p.add(0, 0, 0, 0, -g0.U[0]);
    Poly<T> s2;
    for (int d = 0; d < D; ++d) {
      Poly<T> cd;
      int e[3] = {0, 0, 0};
      e[d] = 1;
      cd.add(e[0], e[1], e[2], 0, T(1.0));
      cd.add(0, 0, 0, 0, -g0.U[d]);
      s2.add(mul(cd, cd), T(0.5));
    }
    s2.add(0, 0, 0, 1, T(0.5));
    w[nc] = mul(c1p, s2);
  }
  const int nw = ns ? nc + 1 : nc;

  // Moments of the three parts of Eq. 2.5.
  T V0[6][3], Vl[6][3], Vr[6][3];
  for (int a = 0; a < nw; ++a) {
    V0[a][0] = g0.mom(w[a]);
    V0[a][1] = g0.mom(mul(w[a], ua0));
    V0[a][2] = g0.mom(mul(w[a], pAb));
    Vl[a][0] = hl.mom(w[a]);
    Vl[a][1] = hl.mom(mul(w[a], ual));
    Vl[a][2] = hl.mom(mul(w[a], pAl));
    Vr[a][0] = hr.mom(w[a]);
    Vr[a][1] = hr.mom(mul(w[a], uar));
    Vr[a][2] = hr.mom(mul(w[a], pAr));
  }
  for (int id = 0; id < ndelta; ++id) {
    const double dl = delta[id];
    // exact time integrals over [0, delta] of the factors in Eq. 2.5
    T e, ome;  // exp(-delta/tau), 1 - exp(-delta/tau)
    if (val(tau) == 0.0) {
      e = T(0.0);
      ome = T(1.0);
    } else {
      e = exp(-dl / tau);
      ome = -expm1(-dl / tau);
    }
    const T C1 = dl - tau * ome;
    const T C2 = 2.0 * tau * tau * ome - tau * dl * (1.0 + e);
    const T C3 = 0.5 * dl * dl - tau * dl + tau * tau * ome;
    const T C4 = tau * ome;
    const T C5 = tau * dl * e - 2.0 * tau * tau * ome;
    const T C6 = -tau * tau * ome;
    T Fa[6];
    for (int a = 0; a < nw; ++a) {
      Fa[a] = g0.rho * ((C1 * V0[a][0] + C2 * V0[a][1]) + C3 * V0[a][2]) +
              hl.rho * ((C4 * Vl[a][0] + C5 * Vl[a][1]) + C6 * Vl[a][2]) +
              hr.rho * ((C4 * Vr[a][0] + C5 * Vr[a][1]) + C6 * Vr[a][2]);
    }
    if (ns) Fa[nc - 1] += (1.0 / P.prandtl - 1.0) * Fa[nc];
    for (int a = 0; a < nc; ++a) F[id][a] = Fa[a];
  }
  return bad;
}

// Equilibrium state of two reconstructed states by kinetic weighting
// (Eq. 2.6): rho_l <psi>_{u>0} + rho_r <psi>_{u<0}, face frame.  Returns 1
// when a state is non-physical.
template <class T>
static int kinetic_w0(const orc_params& P, int D, const T* Wl, const T* Wr, T* W0) {
  const double K = 2.0 / (P.gamma - 1.0) - D;
  Maxw<T> hl, hr;
  hl.build(D, K, Wl, +1);
  hr.build(D, K, Wr, -1);
  for (int a = 0; a < D + 2; ++a) {
    const Poly<T> pa = psi<T>(D, a);
    W0[a] = hl.rho * hl.mom(pa) + hr.rho * hr.mom(pa);
  }
  return state_ok(val(hl.rho), val(hl.pressure())) && state_ok(val(hr.rho), val(hr.pressure())) ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Grid access with boundary conditions (ghost cells by an index map).
// ---------------------------------------------------------------------------
struct Grid {
  int D, nc;
  long n[3];
  long ncell;
  double dx[3];
  int bclo[3], bchi[3];
  const orc_params* P;
  double time;  // time of the prescribed boundary states
  explicit Grid(const orc_params& Pin, double t = 0.0) : P(&Pin), time(t) {
    D = Pin.ndim;
    nc = D + 2;
    ncell = 1;
    for (int d = 0; d < 3; ++d) {
      n[d] = d < D ? Pin.n[d] : 1;
      dx[d] = d < D ? Pin.dx[d] : 1.0;
      bclo[d] = Pin.bc_lo[d];
      bchi[d] = Pin.bc_hi[d];
      ncell *= n[d];
    }
  }
  // map index i along axis d into the interior with the boundary kinds
  // (lo, hi); *flip = 1 behind a reflective wall (the momentum normal to it
  // changes sign), 2 behind a no-slip adiabatic wall (every momentum
  // component changes sign).
  long map(int d, long i, int* flip, int lo, int hi) const {
    const long N = n[d];
    if (d >= D) return 0;
    if (i >= 0 && i < N) return i;
    const int bc = i < 0 ? lo : hi;
    if (bc == 0) return ((i % N) + N) % N;
    if (bc == 1) return i < 0 ? 0 : N - 1;
    *flip ^= bc == 3 ? 2 : 1;
    return i < 0 ? -1 - i : 2 * N - 1 - i;
  }
  long map(int d, long i, int* flip) const { return map(d, i, flip, bclo[d], bchi[d]); }
  long lin(long i, long j, long k) const { return (k * n[1] + j) * n[0] + i; }
};

template <class T>
static T cell(const Grid& g, const T* W, int c, const long idx[3]) {
  int lo[3] = {g.bclo[0], g.bclo[1], g.bclo[2]};
  int hi[3] = {g.bchi[0], g.bchi[1], g.bchi[2]};
  // prescribed sides: the state at the ghost cell's centre
  for (int d = 0; d < g.D && g.D <= 2; ++d) {
    const int e = idx[d] < 0 ? 0 : (idx[d] >= g.n[d] ? 1 : -1);
    if (e < 0 || (e == 0 ? lo[d] : hi[d]) != 4) continue;
    const double s = g.D == 2 ? ((double)idx[1 - d] + 0.5) * g.dx[1 - d] : 0.0;
    const double r = ((double)idx[d] + 0.5) * g.dx[d];
    const double* L = g.P->bc_line[d][e];
    if (s < (L[0] + L[1] * r) + L[2] * g.time) return T(g.P->bc_state[0][c]);
    const int far = g.P->bc_far[d][e];
    if (far == 4) return T(g.P->bc_state[1][c]);
    (e == 0 ? lo[d] : hi[d]) = far;
  }
  int fl[3] = {0, 0, 0};
  long m[3];
  for (int d = 0; d < 3; ++d) m[d] = g.map(d, idx[d], &fl[d], lo[d], hi[d]);
  T v = W[c * g.ncell + g.lin(m[0], m[1], m[2])];
  if (c >= 1 && c <= g.D) {
    bool neg = fl[c - 1] == 1;
    for (int d = 0; d < g.D; ++d) neg ^= fl[d] == 2;
    if (neg) v = -v;
  }
  return v;
}

// Normal TENO-D reconstruction of cell idx along axis d for global component c.
template <class T>
static uint8_t normal_recon(const orc_params& P, const Grid& g, const T* W, int d, int c,
                            const long idx[3], T out[4]) {
  T Q[5];
  for (int r = -2; r <= 2; ++r) {
    long j[3] = {idx[0], idx[1], idx[2]};
    j[d] += r;
    Q[r + 2] = cell(g, W, c, j);
  }
  return recon_face(P, Q, out);
}

// ---------------------------------------------------------------------------
// Characteristic-variable reconstruction (an option; the paper reconstructs
// the conservative variables).  At a face the reference state is the mean of
// the conservative states of the two adjacent cells; the characteristic
// fields are the eigenvectors of the Euler flux Jacobian dF_a/dW along frame
// axis a at that state (a = 0: the face normal, for the normal
// reconstruction; a = 1: along the face, for the tangential one).  Fields,
// in order: u_a - c, entropy, one shear wave per other axis (increasing
// axis), u_a + c.  With u = m / rho, q2 = |u|^2, p = (gamma-1)(E - rho q2/2),
// c^2 = gamma p / rho, H = (E + p) / rho, b1 = (gamma-1)/c^2, b2 = b1 q2 / 2:
//   l(u_a -+ c) = ((b2 +- u_a/c)/2, -(b1 u + -+ e_a / c)/2 ..., b1/2)
//   l(entropy)  = (1 - b2, b1 u, -b1),   l(shear s) = (-u_s, e_s, 0)
//   r(u_a -+ c) = (1, u -+ c e_a, H -+ u_a c), r(entropy) = (1, u, q2/2),
//   r(shear s)  = (0, e_s, u_s).
// Every entry, projection and back-projection follows one fixed operation
// order (dense left-to-right sums over all components), so that identical
// inputs give identical characteristic values and stencil flags.  A
// non-physical reference state (rho <= 0, p <= 0, not finite) falls back to
// the identity (component-wise reconstruction) for that face.
// ---------------------------------------------------------------------------
template <class T>
static bool char_basis(int D, double gamma, const T* Wb, int a, T L[5][5], T R[5][5]) {
  const int nc = D + 2;
  const T rho = Wb[0];
  const T irho = 1.0 / rho;
  T u[3] = {T(0.0), T(0.0), T(0.0)};
  for (int e = 0; e < D; ++e) u[e] = Wb[1 + e] * irho;
  T q2 = u[0] * u[0];
  for (int e = 1; e < D; ++e) q2 = q2 + u[e] * u[e];
  const T E = Wb[D + 1];
  const T p = (gamma - 1.0) * (E - 0.5 * (rho * q2));
  const T c2 = (gamma * p) * irho;
  const bool ok = val(rho) > 0.0 && val(p) > 0.0 && std::isfinite(val(c2)) && std::isfinite(val(E));
  if (!ok) {
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) L[i][j] = R[i][j] = T(i == j ? 1.0 : 0.0);
    return false;
  }
  const T c = sqrt(c2);
  const T ic = 1.0 / c;
  const T H = (E + p) * irho;
  const T b1 = (gamma - 1.0) / c2;
  const T b2 = 0.5 * (b1 * q2);
  const T un = u[a];
  const T uc = un * c;
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) L[i][j] = R[i][j] = T(0.0);
  const int kp = D + 1;  // field u_a + c
  // acoustic rows
  L[0][0] = 0.5 * (b2 + un * ic);
  L[kp][0] = 0.5 * (b2 - un * ic);
  for (int e = 0; e < D; ++e) {
    if (e == a) {
      L[0][1 + e] = 0.5 * (-(b1 * un) - ic);
      L[kp][1 + e] = 0.5 * (ic - b1 * un);
    } else {
      L[0][1 + e] = 0.5 * (-(b1 * u[e]));
      L[kp][1 + e] = 0.5 * (-(b1 * u[e]));
    }
  }
  L[0][D + 1] = 0.5 * b1;
  L[kp][D + 1] = 0.5 * b1;
  // entropy row
  L[1][0] = 1.0 - b2;
  for (int e = 0; e < D; ++e) L[1][1 + e] = b1 * u[e];
  L[1][D + 1] = -b1;
  // shear rows
  int k = 2;
  for (int s = 0; s < D; ++s) {
    if (s == a) continue;
    L[k][0] = -u[s];
    L[k][1 + s] = T(1.0);
    R[1 + s][k] = T(1.0);
    R[D + 1][k] = u[s];
    ++k;
  }
  // right eigenvectors (columns)
  R[0][0] = T(1.0);
  R[0][1] = T(1.0);
  R[0][kp] = T(1.0);
  for (int e = 0; e < D; ++e) {
    R[1 + e][0] = e == a ? un - c : u[e];
    R[1 + e][1] = u[e];
    R[1 + e][kp] = e == a ? un + c : u[e];
  }
  R[D + 1][0] = H - uc;
  R[D + 1][1] = 0.5 * q2;
  R[D + 1][kp] = H + uc;
  return true;
}

// y = M x, dense left-to-right sums
template <class T>
static void matvec(int nc, const T M[5][5], const T* x, T* y) {
  for (int i = 0; i < nc; ++i) {
    T v = M[i][0] * x[0];
    for (int j = 1; j < nc; ++j) v = v + M[i][j] * x[j];
    y[i] = v;
  }
}

// density and pressure of a frame-ordered state positive and finite (the
// test of the first-order fallback, in one fixed operation order)
template <class T>
static bool physical_state(int D, double gamma, const T* w) {
  T ke = T(0.0);
  for (int a = 1; a <= D; ++a) ke = ke + w[a] * w[a];
  const T pr = (gamma - 1.0) * (w[D + 1] - 0.5 * ke / w[0]);
  return val(w[0]) > 0.0 && val(pr) > 0.0 && std::isfinite(val(w[0])) && std::isfinite(val(pr));
}

// conservative state of a cell in frame order
template <class T>
static void cell_frame(const Grid& g, const T* W, const int* perm, const long idx[3], T* out) {
  for (int a = 0; a < g.nc; ++a) out[a] = cell(g, W, perm[a], idx);
}

// Normal reconstruction of both sides of a face in characteristic
// variables from the six frame-ordered cells C[0..5] = cells f-3 .. f+2
// along the normal: values and slopes (per unit length, idn = 1/dx) in frame
// order; fr = flags of the right side (cell f at its low face).
template <class T>
static void char_recon_cells(const orc_params& P, int D, const T C[6][5], double idn, T vl[5], T sl[5],
                             T vr[5], T sr[5], uint8_t fr[5]) {
  const int nc = D + 2;
  T Wb[5], L[5][5], R[5][5];
  for (int a = 0; a < 5; ++a) Wb[a] = a < nc ? 0.5 * (C[2][a] + C[3][a]) : T(0.0);
  char_basis(D, P.gamma, Wb, 0, L, R);
  T V[6][5];
  for (int r = 0; r < 6; ++r) matvec(nc, L, C[r], V[r]);
  T ol[5][4], orr[5][4];
  for (int k = 0; k < nc; ++k) {
    T Ql[5], Qr[5];
    for (int r = 0; r < 5; ++r) {
      Ql[r] = V[r][k];
      Qr[r] = V[r + 1][k];
    }
    const uint8_t f0 = select_T(Ql, P.ct1, P.ct2, P.eps, P.q);
    const uint8_t f1 = select_T(Qr, P.ct1, P.ct2, P.eps, P.q);
    teno_face_values(Ql, f0, ol[k]);
    teno_face_values(Qr, f1, orr[k]);
    fr[k] = f1;
  }
  T a[5] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
  for (int k = 0; k < nc; ++k) a[k] = ol[k][2];
  matvec(nc, R, a, vl);
  for (int k = 0; k < nc; ++k) a[k] = ol[k][3];
  matvec(nc, R, a, sl);
  for (int k = 0; k < nc; ++k) a[k] = orr[k][0];
  matvec(nc, R, a, vr);
  for (int k = 0; k < nc; ++k) a[k] = orr[k][1];
  matvec(nc, R, a, sr);
  for (int q = 0; q < nc; ++q) {
    sl[q] = sl[q] * idn;
    sr[q] = sr[q] * idn;
  }
}

// the same for the face at fpos of direction d of the grid
template <class T>
static void char_normal_face(const orc_params& P, const Grid& g, const T* W, int d, const int* perm,
                             const long fpos[3], T vl[5], T sl[5], T vr[5], T sr[5], uint8_t fr[5]) {
  T C[6][5];
  for (int r = 0; r < 6; ++r) {
    long j[3] = {fpos[0], fpos[1], fpos[2]};
    j[d] += r - 3;
    cell_frame(g, W, perm, j, C[r]);
  }
  char_recon_cells(P, g.D, C, 1.0 / g.dx[d], vl, sl, vr, sr, fr);
}

// Face-averaged fluxes over every face of direction d for the intervals
// dt and dt/2, global component order, layout [nc][faces] with faces indexed
// with the direction-d face index in place of the cell index.
template <class T>
static long face_fluxes(const orc_params& P, const Grid& g, const T* W, int d, double dt,
                        std::vector<T>& Fdt, std::vector<T>& Fh, uint8_t* nflags,
                        uint8_t* tflags, long* nfallback = nullptr) {
  const int D = g.D, nc = g.nc;
  long nf[3] = {g.n[0], g.n[1], g.n[2]};
  nf[d] += 1;
  const long nface = nf[0] * nf[1] * nf[2];
  Fdt.assign((size_t)nc * nface, T(0.0));
  Fh.assign((size_t)nc * nface, T(0.0));
  const int t1 = D >= 2 ? (d + 1) % D : -1;
  const int t2 = D == 3 ? (d + 2) % D : -1;
  // frame component a -> global component
  int perm[5];
  perm[0] = 0;
  perm[1] = 1 + d;
  if (D >= 2) perm[2] = 1 + t1;
  if (D == 3) perm[3] = 1 + t2;
  perm[D + 1] = D + 1;
  const double dn = g.dx[d];
  const double idn = 1.0 / dn;  // normal slopes per unit length
  const double dt1 = t1 >= 0 ? g.dx[t1] : 1.0, dt2 = t2 >= 0 ? g.dx[t2] : 1.0;
  const double deltas[2] = {dt, 0.5 * dt};
  long nbad = 0, nfb = 0;

#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nbad, nfb)
  for (long fidx = 0; fidx < nface; ++fidx) {
    long fpos[3];
    fpos[0] = fidx % nf[0];
    fpos[1] = (fidx / nf[0]) % nf[1];
    fpos[2] = fidx / (nf[0] * nf[1]);
    // cells on the left (f-1) and right (f) of this face
    long cl[3] = {fpos[0], fpos[1], fpos[2]}, cr[3] = {fpos[0], fpos[1], fpos[2]};
    cl[d] -= 1;
    const int ngp1 = D >= 2 ? 2 : 1, ngp2 = D == 3 ? 2 : 1;
    const double wgp = 1.0 / (ngp1 * ngp2);
    // per Gauss point, per side: W, dW/dn, dW/dt1, dW/dt2 in frame order
    T Wg[2][2][2][5], Dg[2][2][2][3][5];
    // WENO-Z / TENO5 (2-D): the line-averaged interface values of the five
    // face segments of the tangential stencil, [side][row][frame component]
    T Lrow[2][5][5];
    if (P.recon == 1) {
      if (D == 1) {
        T vl[5], sl[5], vr[5], sr[5];
        uint8_t fr[5];
        char_normal_face(P, g, W, d, perm, fpos, vl, sl, vr, sr, fr);
        if (nflags && fpos[d] < g.n[d])
          for (int k = 0; k < nc; ++k) nflags[(long)d * nc * g.ncell + (long)k * g.ncell + g.lin(fpos[0], fpos[1], fpos[2])] = fr[k];
        for (int a = 0; a < nc; ++a) {
          Wg[0][0][0][a] = vl[a];
          Dg[0][0][0][0][a] = sl[a];
          Wg[0][0][1][a] = vr[a];
          Dg[0][0][1][0][a] = sr[a];
        }
      } else {
        // normal reconstruction (each face of the tangential stencil in its
        // own normal basis), then the tangential one in the basis along the
        // face at this face's reference state
        T X[2][5][5], Xn[2][5][5];  // [side][r][frame component]
        for (int r = -2; r <= 2; ++r) {
          long j[3] = {fpos[0], fpos[1], fpos[2]};
          j[t1] += r;
          T vl[5], sl[5], vr[5], sr[5];
          uint8_t fr[5];
          char_normal_face(P, g, W, d, perm, j, vl, sl, vr, sr, fr);
          if (r == 0 && nflags && fpos[d] < g.n[d])
            for (int k = 0; k < nc; ++k) nflags[(long)d * nc * g.ncell + (long)k * g.ncell + g.lin(fpos[0], fpos[1], fpos[2])] = fr[k];
          for (int a = 0; a < nc; ++a) {
            X[0][r + 2][a] = vl[a];
            Xn[0][r + 2][a] = sl[a];
            X[1][r + 2][a] = vr[a];
            Xn[1][r + 2][a] = sr[a];
          }
        }
        T Cl[5], Cr[5], Wb[5], L[5][5], R[5][5];
        cell_frame(g, W, perm, cl, Cl);
        cell_frame(g, W, perm, cr, Cr);
        for (int a = 0; a < nc; ++a) Wb[a] = 0.5 * (Cl[a] + Cr[a]);
        char_basis(D, P.gamma, Wb, 1, L, R);
        for (int side = 0; side < 2; ++side) {
          T ow[5][4], on[5][4];
          for (int qn = 0; qn < 2; ++qn) {
            T Vr[5][5];  // [r][field]
            for (int r = 0; r < 5; ++r) matvec(nc, L, qn == 0 ? X[side][r] : Xn[side][r], Vr[r]);
            for (int k = 0; k < nc; ++k) {
              T Q[5];
              for (int r = 0; r < 5; ++r) Q[r] = Vr[r][k];
              const uint8_t f = select_T(Q, P.ct1_tan, P.ct2_tan, P.eps, P.q);
              if (tflags) tflags[(((long)qn * 2 + side) * nc + k) * nface + fidx] = f;
              teno_gauss_values(Q, f, qn == 0 ? ow[k] : on[k]);
            }
          }
          for (int m = 0; m < 2; ++m) {
            T a[5], b[5];
            for (int k = 0; k < nc; ++k) a[k] = ow[k][2 * m];
            matvec(nc, R, a, b);
            for (int q = 0; q < nc; ++q) Wg[m][0][side][q] = b[q];
            for (int k = 0; k < nc; ++k) a[k] = ow[k][2 * m + 1];
            matvec(nc, R, a, b);
            for (int q = 0; q < nc; ++q) Dg[m][0][side][1][q] = b[q] / dt1;
            for (int k = 0; k < nc; ++k) a[k] = on[k][2 * m];
            matvec(nc, R, a, b);
            for (int q = 0; q < nc; ++q) Dg[m][0][side][0][q] = b[q];
          }
        }
      }
    }
    for (int side = 0; side < 2 && P.recon != 1; ++side) {
      const long* cc = side == 0 ? cl : cr;
      const int vo = side == 0 ? 2 : 0;  // +1/2 values of the left cell, -1/2 of the right
      for (int a = 0; a < nc; ++a) {
        const int c = perm[a];
        if (D == 1) {
          T o[4];
          const uint8_t f = normal_recon(P, g, W, d, c, cc, o);
          if (side == 1 && nflags && cc[d] < g.n[d]) nflags[(long)d * nc * g.ncell + (long)c * g.ncell + g.lin(cc[0], cc[1], cc[2])] = f;
          Wg[0][0][side][a] = o[vo];
          Dg[0][0][side][0][a] = o[vo + 1] * idn;
        } else if (D == 2) {
          T Wl[5], Nl[5];
          for (int r = -2; r <= 2; ++r) {
            long j[3] = {cc[0], cc[1], cc[2]};
            j[t1] += r;
            T o[4];
            const uint8_t f = normal_recon(P, g, W, d, c, j, o);
            if (r == 0 && side == 1 && nflags && cc[d] < g.n[d])
              nflags[(long)d * nc * g.ncell + (long)c * g.ncell + g.lin(cc[0], cc[1], cc[2])] = f;
            Wl[r + 2] = o[vo];
            Nl[r + 2] = o[vo + 1] * idn;
          }
          T ow[4], on[4];
          const uint8_t fw = recon_gauss(P, Wl, ow);
          const uint8_t fn = recon_gauss(P, Nl, on);
          if (tflags) {
            // layout per direction: [(q*2 + side)*nc + c][face], q = 0 (W), 1 (W_n)
            tflags[(((long)0 * 2 + side) * nc + c) * nface + fidx] = fw;
            tflags[(((long)1 * 2 + side) * nc + c) * nface + fidx] = fn;
          }
          if (P.scheme >= 2)
            for (int r = 0; r < 5; ++r) Lrow[side][r][a] = Wl[r];
          for (int m = 0; m < 2; ++m) {
            Wg[m][0][side][a] = ow[2 * m];
            Dg[m][0][side][1][a] = ow[2 * m + 1] / dt1;
            Dg[m][0][side][0][a] = on[2 * m];
          }
        } else {
          // 3-D: normal values on the 5x5 tangential patch, sweep along t1
          // at every t2 offset, then along t2.
          T Vw[5][5], Vn[5][5];
          for (int r2 = -2; r2 <= 2; ++r2)
            for (int r1 = -2; r1 <= 2; ++r1) {
              long j[3] = {cc[0], cc[1], cc[2]};
              j[t1] += r1;
              j[t2] += r2;
              T o[4];
              const uint8_t f = normal_recon(P, g, W, d, c, j, o);
              if (r1 == 0 && r2 == 0 && side == 1 && nflags && cc[d] < g.n[d])
                nflags[(long)d * nc * g.ncell + (long)c * g.ncell + g.lin(cc[0], cc[1], cc[2])] = f;
              Vw[r2 + 2][r1 + 2] = o[vo];
              Vn[r2 + 2][r1 + 2] = o[vo + 1] * idn;
            }
          T S1w[2][5], S1d[2][5], S1n[2][5];  // [m1][r2]
          for (int r2 = 0; r2 < 5; ++r2) {
            const uint8_t fw = select_T(Vw[r2], P.ct1_tan, P.ct2_tan, P.eps, P.q);
            const uint8_t fn = select_T(Vn[r2], P.ct1_tan, P.ct2_tan, P.eps, P.q);
            if (tflags && r2 == 2) {
              // sweep 1 of the face's own line: [(q*2 + side)*nc + c][face],
              // q = 0 (W), 1 (W_n)
              tflags[(((long)0 * 2 + side) * nc + c) * nface + fidx] = fw;
              tflags[(((long)1 * 2 + side) * nc + c) * nface + fidx] = fn;
            }
            T ow[4], on[4];
            teno_gauss_canonical(Vw[r2], fw, ow);
            teno_gauss_canonical(Vn[r2], fn, on);
            for (int m1 = 0; m1 < 2; ++m1) {
              S1w[m1][r2] = ow[2 * m1];
              // scaled by the reciprocal width, like every slope that a
              // later selection takes as input (one rounding order)
              S1d[m1][r2] = ow[2 * m1 + 1] * (1.0 / dt1);
              S1n[m1][r2] = on[2 * m1];
            }
          }
          for (int m1 = 0; m1 < 2; ++m1) {
            const uint8_t fw = select_T(S1w[m1], P.ct1_tan, P.ct2_tan, P.eps, P.q);
            const uint8_t fd = select_T(S1d[m1], P.ct1_tan, P.ct2_tan, P.eps, P.q);
            const uint8_t fn = select_T(S1n[m1], P.ct1_tan, P.ct2_tan, P.eps, P.q);
            if (tflags) {
              // sweep 2 at t1 Gauss point m1: [4 nc + ((m1*3 + kind)*2 + side)*nc
              // + c][face], kind 0 (W), 1 (dW/dt1), 2 (W_n)
              const uint8_t fk[3] = {fw, fd, fn};
              for (int kind = 0; kind < 3; ++kind)
                tflags[(4L * nc + ((long)(m1 * 3 + kind) * 2 + side) * nc + c) * nface + fidx] = fk[kind];
            }
            T ow[4], od[4], on[4];
            teno_gauss_values(S1w[m1], fw, ow);
            teno_gauss_values(S1d[m1], fd, od);
            teno_gauss_values(S1n[m1], fn, on);
            for (int m2 = 0; m2 < 2; ++m2) {
              Wg[m1][m2][side][a] = ow[2 * m2];
              Dg[m1][m2][side][2][a] = ow[2 * m2 + 1] / dt2;
              Dg[m1][m2][side][1][a] = od[2 * m2];
              Dg[m1][m2][side][0][a] = on[2 * m2];
            }
          }
        }
      }
    }
    T acc[2][5];
    for (int i = 0; i < 2; ++i)
      for (int a = 0; a < 5; ++a) acc[i][a] = T(0.0);
    if (P.fallback) {
      // first-order fallback: a non-physical side state at a Gauss point
      // becomes the side's cell average with zero slopes
      T C[2][5];
      cell_frame(g, W, perm, cl, C[0]);
      cell_frame(g, W, perm, cr, C[1]);
      for (int m1 = 0; m1 < ngp1; ++m1)
        for (int m2 = 0; m2 < ngp2; ++m2)
          for (int side = 0; side < 2; ++side) {
            T* w = Wg[m1][m2][side];
            if (physical_state(D, P.gamma, w)) continue;
            ++nfb;
            for (int a = 0; a < nc; ++a) {
              w[a] = C[side][a];
              for (int q = 0; q < 3; ++q) Dg[m1][m2][side][q][a] = T(0.0);
            }
          }
    }
    // WENO-Z / TENO5: the equilibrium state's slopes (and in 2-D its value)
    // are reconstructed separately (Sec. 3.1): along the normal by the
    // fifth-order linear formula of Eq. 3.12 on each face segment, whose
    // equilibrium value is the kinetic weighting of its line-averaged
    // interface values (Eq. 2.6); along the face (Steps 2 and 4) by the
    // fifth-order reconstruction of the five segments at the Gauss points
    // with the ENO-like cut-off of Sec. 4.1 (TENO5, q = 6): the linear
    // quartic wherever the segments' states are smooth (Tables 5 and 7),
    // without its overshoot at a discontinuity, where the unlimited quartic
    // gives non-physical equilibrium states in the first step of the 2-D
    // Riemann problems the paper runs both schemes on (Sec. 5.6)
    T E0[2][5], dE0[2][3][5];
    const bool sep = P.scheme >= 2;
    if (sep) {
      const int nrow = D == 2 ? 5 : 1;
      T W0row[5][5], W0xrow[5][5];
      for (int r = 0; r < nrow; ++r) {
        const int rr = D == 2 ? r - 2 : 0;
        T Wl_[5], Wr_[5];
        for (int a = 0; a < nc; ++a) {
          Wl_[a] = D == 2 ? Lrow[0][r][a] : Wg[0][0][0][a];
          Wr_[a] = D == 2 ? Lrow[1][r][a] : Wg[0][0][1][a];
        }
        // a non-physical segment state shows as a non-physical equilibrium
        // at the Gauss points, counted there
        (void)kinetic_w0(P, D, Wl_, Wr_, W0row[r]);
        for (int a = 0; a < nc; ++a) {
          T q[4];
          for (int k = 0; k < 4; ++k) {
            long j[3] = {cl[0], cl[1], cl[2]};
            j[d] += k - 1;
            if (D == 2) j[t1] += rr;
            q[k] = cell(g, W, perm[a], j);
          }
          // cells f-2, f-1, f, f+1 along the normal (Eq. 3.12)
          W0xrow[r][a] = ((-1.0 / 12.0) * (q[3] - q[0]) + 1.25 * (q[2] - q[1])) * idn;
        }
      }
      for (int m = 0; m < ngp1; ++m)
        for (int a = 0; a < nc; ++a) {
          if (D == 1) {
            E0[m][a] = W0row[0][a];
            dE0[m][0][a] = W0xrow[0][a];
            continue;
          }
          T Qv[5], Qx[5], ov[4], ox[4];
          for (int r = 0; r < 5; ++r) {
            Qv[r] = W0row[r][a];
            Qx[r] = W0xrow[r][a];
          }
          orc_params Pe = P;  // the cut-off reconstruction of Sec. 4.1 (TENO5)
          Pe.scheme = 2;
          Pe.q = 6;
          scheme_gauss(Pe, Qv, ov);
          scheme_gauss(Pe, Qx, ox);
          E0[m][a] = ov[2 * m];
          dE0[m][1][a] = ov[2 * m + 1] / dt1;
          dE0[m][0][a] = ox[2 * m];
        }
    }
    for (int m1 = 0; m1 < ngp1; ++m1)
      for (int m2 = 0; m2 < ngp2; ++m2) {
        T F[2][5];
        nbad += gp_flux(P, D, Wg[m1][m2][0], Wg[m1][m2][1], Dg[m1][m2][0], Dg[m1][m2][1], dt, 2,
                        deltas, F, (T*)nullptr, (T(*)[5]) nullptr, sep && D == 2 ? E0[m1] : (const T*)nullptr,
                        sep ? dE0[m1] : (const T(*)[5]) nullptr);
        for (int i = 0; i < 2; ++i)
          for (int a = 0; a < nc; ++a) acc[i][a] += wgp * F[i][a];
      }
    // a no-slip adiabatic wall is impermeable and, at rest, does no work
    // and conducts no heat: no mass or energy crosses it
    const bool wall = (fpos[d] == 0 && g.bclo[d] == 3) || (fpos[d] == g.n[d] && g.bchi[d] == 3);
    if (wall)
      for (int i = 0; i < 2; ++i) acc[i][0] = acc[i][nc - 1] = T(0.0);
    for (int a = 0; a < nc; ++a) {
      Fdt[(size_t)perm[a] * nface + fidx] = acc[0][a];
      Fh[(size_t)perm[a] * nface + fidx] = acc[1][a];
    }
  }
  if (nfallback) *nfallback += nfb;
  return nbad;
}

// index of the face on the low (s=0) or high (s=1) side of cell (i,j,k) along d
static inline long face_index(const Grid& g, int d, long i, long j, long k, int s) {
  long nf[3] = {g.n[0], g.n[1], g.n[2]};
  nf[d] += 1;
  long p[3] = {i, j, k};
  p[d] += s;
  return (p[2] * nf[1] + p[1]) * nf[0] + p[0];
}

// One S2O4 step (Sec. 2.2).
template <class T>
static long s2o4_step(const orc_params& P, const T* Wn, T* Wout, double dt, uint8_t* flags,
                      T* Wstar_out, double t = 0.0, long* nfallback = nullptr) {
  const Grid g(P, t);
  const Grid gs(P, t + 0.5 * dt);  // stage 2: W* is the state at the half step
  const int D = g.D, nc = g.nc;
  const long N = g.ncell;
  long nbad = 0;
  std::vector<T> Fdt[3], Fh[3], Gdt[3], Gh[3];
  // flag layout: normal [D][nc][cells], then tangential per direction
  // (2-D: 4 nc planes of faces; 3-D: 4 nc of sweep 1 and 12 nc of sweep 2)
  uint8_t* tfl[3] = {nullptr, nullptr, nullptr};
  if (flags && D >= 2) {
    long off = (long)D * nc * N;
    for (int d = 0; d < D; ++d) {
      long nf[3] = {g.n[0], g.n[1], g.n[2]};
      nf[d] += 1;
      tfl[d] = flags + off;
      off += (D == 2 ? 4L : 16L) * nc * nf[0] * nf[1] * nf[2];
    }
  }
  for (int d = 0; d < D; ++d) nbad += face_fluxes(P, g, Wn, d, dt, Fdt[d], Fh[d], flags, tfl[d], nfallback);
  // F^n = (4 F(dt/2) - F(dt)) / dt,  d_t F^n = 4 (F(dt) - 2 F(dt/2)) / dt^2
  std::vector<T> Fn[3], dFn[3];
  for (int d = 0; d < D; ++d) {
    Fn[d].resize(Fdt[d].size());
    dFn[d].resize(Fdt[d].size());
    for (size_t i = 0; i < Fdt[d].size(); ++i) {
      Fn[d][i] = (4.0 * Fh[d][i] - Fdt[d][i]) / dt;
      dFn[d][i] = 4.0 * (Fdt[d][i] - 2.0 * Fh[d][i]) / (dt * dt);
    }
  }
  // W* = W^n - sum_d (1/dx_d) [F(W^n, dt/2)_{+} - F(W^n, dt/2)_{-}]
  std::vector<T> Ws((size_t)nc * N);
  for (long k = 0; k < g.n[2]; ++k)
    for (long j = 0; j < g.n[1]; ++j)
      for (long i = 0; i < g.n[0]; ++i) {
        const long id = g.lin(i, j, k);
        for (int c = 0; c < nc; ++c) {
          T v = Wn[(size_t)c * N + id];
          for (int d = 0; d < D; ++d) {
            long nf[3] = {g.n[0], g.n[1], g.n[2]};
            nf[d] += 1;
            const long nface = nf[0] * nf[1] * nf[2];
            (void)nface;
            const T fp = Fh[d][(size_t)c * nface + face_index(g, d, i, j, k, 1)];
            const T fm = Fh[d][(size_t)c * nface + face_index(g, d, i, j, k, 0)];
            v -= (fp - fm) / g.dx[d];
          }
          Ws[(size_t)c * N + id] = v;
        }
      }
  if (Wstar_out)
    for (size_t i = 0; i < Ws.size(); ++i) Wstar_out[i] = Ws[i];
  for (int d = 0; d < D; ++d)
    nbad += face_fluxes(P, gs, Ws.data(), d, dt, Gdt[d], Gh[d], (uint8_t*)nullptr, (uint8_t*)nullptr, nfallback);
  // combined flux F^n + dt/6 (d_tF^n + 2 d_tF*), then the final update
  std::vector<T> Fc[3];
  for (int d = 0; d < D; ++d) {
    Fc[d].resize(Fdt[d].size());
    for (size_t i = 0; i < Fdt[d].size(); ++i) {
      const T dFs = 4.0 * (Gdt[d][i] - 2.0 * Gh[d][i]) / (dt * dt);
      Fc[d][i] = Fn[d][i] + (dt / 6.0) * (dFn[d][i] + 2.0 * dFs);
    }
  }
  for (long k = 0; k < g.n[2]; ++k)
    for (long j = 0; j < g.n[1]; ++j)
      for (long i = 0; i < g.n[0]; ++i) {
        const long id = g.lin(i, j, k);
        for (int c = 0; c < nc; ++c) {
          T v = Wn[(size_t)c * N + id];
          for (int d = 0; d < D; ++d) {
            long nf[3] = {g.n[0], g.n[1], g.n[2]};
            nf[d] += 1;
            const long nface = nf[0] * nf[1] * nf[2];
            const T fp = Fc[d][(size_t)c * nface + face_index(g, d, i, j, k, 1)];
            const T fm = Fc[d][(size_t)c * nface + face_index(g, d, i, j, k, 0)];
            v -= (dt / g.dx[d]) * (fp - fm);
          }
          Wout[(size_t)c * N + id] = v;
        }
      }
  return nbad;
}

// CFL time step (Sec. 5 preamble): C min(dx/(|U| + a), dx^2/(4 nu)).
static double cfl_dt(const orc_params& P, const double* W, double cfl) {
  const Grid g(P);
  const int D = g.D;
  double dxm = g.dx[0];
  for (int d = 1; d < D; ++d) dxm = std::min(dxm, g.dx[d]);
  double best = INFINITY;
  bool nan = false;
  for (long id = 0; id < g.ncell; ++id) {
    const double rho = W[id];
    double ke = 0.0;
    for (int d = 0; d < D; ++d) {
      const double u = W[(size_t)(1 + d) * g.ncell + id] / rho;
      ke += u * u;
    }
    const double p = (P.gamma - 1.0) * (W[(size_t)(D + 1) * g.ncell + id] - 0.5 * rho * ke);
    const double a = std::sqrt(P.gamma * p / rho);
    double v = dxm / (std::sqrt(ke) + a);
    if (P.mu > 0.0) v = std::min(v, dxm * dxm * rho / (4.0 * P.mu));
    if (std::isnan(v)) nan = true;
    best = std::min(best, v);
  }
  return nan ? NAN : cfl * best;
}

static int check_params(const orc_params* P) {
  if (!P || P->ndim < 1 || P->ndim > 3) return -1;
  for (int d = 0; d < P->ndim; ++d) {
    if (P->n[d] < 3 || !(P->dx[d] > 0)) return -1;
    if (P->bc_lo[d] < 0 || P->bc_lo[d] > 4 || P->bc_hi[d] < 0 || P->bc_hi[d] > 4) return -1;
    if ((P->bc_lo[d] == 0) != (P->bc_hi[d] == 0)) return -1;
    for (int e = 0; e < 2; ++e) {
      if ((e == 0 ? P->bc_lo[d] : P->bc_hi[d]) != 4) continue;
      if (P->ndim > 2) return -1;
      const int far = P->bc_far[d][e];
      if (far != 1 && far != 2 && far != 4) return -1;
    }
  }
  if (!(P->gamma > 1.0)) return -1;
  if (P->recon < 0 || P->recon > 1 || (P->recon == 1 && P->ndim > 2)) return -1;
  if (P->fallback < 0 || P->fallback > 1) return -1;
  if (P->scheme < 0 || P->scheme > 3) return -1;
  if (P->scheme != 0) {
    // the comparison schemes: conservative variables on 1-D and 2-D grids
    if (P->ndim > 2 || P->recon != 0 || P->fallback != 0) return -1;
    if (P->scheme == 1 && !(P->d_hi > 0.0 && P->d_hi < 1.0 && P->d_lo > 0.0 && P->d_lo < 1.0)) return -1;
    if ((P->scheme == 1 || P->scheme == 3) && !(P->eps_w > 0.0)) return -1;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// C interface used by oracle/oracle.py.
// ---------------------------------------------------------------------------
extern "C" {

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_beta(const double* Q, double* beta) {
  teno_beta(Q, beta);
  return 0;
}

int orc_teno_select(const double* Q, double ct1, double ct2, double eps, int q) {
  return teno_select(Q, ct1, ct2, eps, q);
}

// out = {v(-1/2), d(-1/2), v(+1/2), d(+1/2)} in cell units; returns the flag.
int orc_teno_face(const double* Q, double ct1, double ct2, double eps, int q, double* out) {
  const uint8_t f = teno_select(Q, ct1, ct2, eps, q);
  teno_face_values(Q, f, out);
  return f;
}

// out = {v(s-), d(s-), v(s+), d(s+)} at s = -+1/(2 sqrt 3); returns the flag.
int orc_teno_gauss(const double* Q, double ct1, double ct2, double eps, int q, double* out) {
  const uint8_t f = teno_select(Q, ct1, ct2, eps, q);
  teno_gauss_values(Q, f, out);
  return f;
}

// Reconstruction of the configured scheme (P->scheme) from five values:
// gauss = 0: {v(-1/2), s(-1/2), v(+1/2), s(+1/2)}, gauss = 1: {v(s-), d(s-),
// v(s+), d(s+)} in cell units; returns the flags (TENO-D, TENO5) or 0.
int orc_recon(const orc_params* P, const double* Q, int gauss, double* out) {
  if (check_params(P)) return -1;
  return gauss ? recon_gauss(*P, Q, out) : recon_face(*P, Q, out);
}

// Linear weights of p_0..p_2 at x = -1/2, +1/2, s-, s+ (where = 0..3).
int orc_lin_weights(int where, double* d) {
  if (where < 0 || where > 3) return -1;
  lin_weights(where, d);
  return 0;
}

// The canonical-order Gauss-point evaluation of the 3-D first sweep with a
// caller-given flag: {v(s-), d(s-), v(s+), d(s+)}.
int orc_teno_gauss_canonical(const double* Q, int flag, double* out) {
  teno_gauss_canonical(Q, (uint8_t)flag, out);
  return 0;
}

// The same with a caller-forced flag (for exactness tests of each candidate).
int orc_teno_eval(const double* Q, int flag, int gauss, double* out) {
  if (gauss)
    teno_gauss_values(Q, (uint8_t)flag, out);
  else
    teno_face_values(Q, (uint8_t)flag, out);
  return 0;
}

int orc_moments(double U, double lam, int kind, double* out) {
  mom1d(U, lam, kind, out);
  return NM;
}

// Micro-slope solve: a with <a psi> = b over the Maxwellian of state W.
int orc_micro_slope(int D, double gamma, const double* W, const double* b, double* a) {
  const double K = 2.0 / (gamma - 1.0) - D;
  Maxw<double> m;
  m.build(D, K, W, 0);
  solve_micro(m, b, a);
  return 0;
}

// Moment of psi_alpha psi_beta u1^e0 u2^e1 u3^e2 xi^(2 e3) per unit density
// over the Maxwellian of W (kind 0 full, +1 u1>0, -1 u1<0).
double orc_moment_mono(int D, double gamma, const double* W, int kind, int e0, int e1, int e2,
                       int e3) {
  const double K = 2.0 / (gamma - 1.0) - D;
  Maxw<double> m;
  m.build(D, K, W, kind);
  const int e[4] = {e0, e1, e2, e3};
  return m.mono(e);
}

// GKS flux at a single Gauss point in the face frame.
// dWl, dWr: [3][5] derivatives (frame axis order), F: [ndelta][5].
int orc_gp_flux(const orc_params* P, const double* Wl, const double* Wr, const double* dWl,
                const double* dWr, double dt, int ndelta, const double* delta, double* F,
                double* W0, double* dW0) {
  if (check_params(P) || ndelta < 1 || ndelta > 2) return -1;
  const int D = P->ndim;
  double a[3][5], b[3][5], Fo[2][5], dw[3][5];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 5; ++c) {
      a[d][c] = dWl[d * 5 + c];
      b[d][c] = dWr[d * 5 + c];
    }
  const int bad = gp_flux(*P, D, Wl, Wr, a, b, dt, ndelta, delta, Fo, W0, dw);
  for (int i = 0; i < ndelta; ++i)
    for (int c = 0; c < D + 2; ++c) F[i * 5 + c] = Fo[i][c];
  if (dW0)
    for (int d = 0; d < D; ++d)
      for (int c = 0; c < D + 2; ++c) dW0[d * 5 + c] = dw[d][c];
  return bad;
}

// Directional derivative of the Gauss-point flux (forward mode, the dual
// type above) along (tWl, tWr, tdWl, tdWr) with dt and the deltas constant:
// F[i*5+c] and dF[i*5+c] for delta i.  Same layout as orc_gp_flux.
int orc_gp_flux_dual(const orc_params* P, const double* Wl, const double* Wr, const double* dWl,
                     const double* dWr, const double* tWl, const double* tWr, const double* tdWl,
                     const double* tdWr, double dt, int ndelta, const double* delta, double* F,
                     double* dF) {
  if (check_params(P) || ndelta < 1 || ndelta > 2) return -1;
  const int D = P->ndim;
  Dual l[5], r[5], a[3][5], b[3][5], Fo[2][5], W0[5], dw[3][5];
  for (int c = 0; c < 5; ++c) {
    l[c] = Dual(Wl[c], tWl[c]);
    r[c] = Dual(Wr[c], tWr[c]);
  }
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 5; ++c) {
      a[d][c] = Dual(dWl[d * 5 + c], tdWl[d * 5 + c]);
      b[d][c] = Dual(dWr[d * 5 + c], tdWr[d * 5 + c]);
    }
  const int bad = gp_flux(*P, D, l, r, a, b, dt, ndelta, delta, Fo, W0, dw);
  for (int i = 0; i < ndelta; ++i)
    for (int c = 0; c < D + 2; ++c) {
      F[i * 5 + c] = Fo[i][c].v;
      dF[i * 5 + c] = Fo[i][c].d;
    }
  return bad;
}

// Characteristic basis along frame axis a at the frame-ordered state Wb:
// L (rows) and R (columns), row-major nc x nc.  Returns 1 for a physical
// state, 0 when the identity was returned.
int orc_char_basis(int D, double gamma, const double* Wb, int a, double* L, double* R) {
  if (D < 1 || D > 3 || a < 0 || a >= D) return -1;
  double l[5][5], r[5][5];
  const bool ok = char_basis(D, gamma, Wb, a, l, r);
  for (int i = 0; i < D + 2; ++i)
    for (int j = 0; j < D + 2; ++j) {
      L[i * (D + 2) + j] = l[i][j];
      R[i * (D + 2) + j] = r[i][j];
    }
  return ok ? 1 : 0;
}

// Characteristic normal reconstruction of one face from six frame-ordered
// cells C (6 x nc) with cell width dx: out = {vl, sl, vr, sr} (4 x nc).
int orc_char_recon(const orc_params* P, const double* C, double dx, double* out, uint8_t* fr) {
  if (!P || P->ndim < 1 || P->ndim > 3) return -1;
  const int nc = P->ndim + 2;
  double c[6][5];
  for (int r = 0; r < 6; ++r)
    for (int a = 0; a < nc; ++a) c[r][a] = C[r * nc + a];
  double vl[5], sl[5], vr[5], sr[5];
  char_recon_cells(*P, P->ndim, c, 1.0 / dx, vl, sl, vr, sr, fr);
  for (int a = 0; a < nc; ++a) {
    out[a] = vl[a];
    out[nc + a] = sl[a];
    out[2 * nc + a] = vr[a];
    out[3 * nc + a] = sr[a];
  }
  return 0;
}

// Number of bytes of the flag buffer of one step: the normal flags, then the
// tangential flags of every direction (2-D: [W, W_n][side][nc][faces]; 3-D:
// sweep 1 of each face's own line as in 2-D, then sweep 2 as
// [t1 Gauss point][W, dW/dt1, W_n][side][nc][faces]).
long orc_flag_bytes(const orc_params* P) {
  if (check_params(P)) return -1;
  const Grid g(*P);
  long nb = (long)g.D * g.nc * g.ncell;
  if (g.D >= 2)
    for (int d = 0; d < g.D; ++d) {
      long nf[3] = {g.n[0], g.n[1], g.n[2]};
      nf[d] += 1;
      nb += (g.D == 2 ? 4L : 16L) * g.nc * nf[0] * nf[1] * nf[2];
    }
  return nb;
}

// One S2O4 step; returns the number of failing Gauss-point evaluations, or -1.
// t: time of W (prescribed boundary states); fallbacks (or null) receives the
// number of Gauss-point side states the first-order fallback replaced, both
// stages.
long orc_step(const orc_params* P, const double* W, double* Wout, double dt, uint8_t* flags,
              double* Wstar, double t, long* fallbacks) {
  if (check_params(P) || !(dt > 0)) return -1;
  long nfb = 0;
  const long bad = s2o4_step<double>(*P, W, Wout, dt, flags, Wstar, t, &nfb);
  if (fallbacks) *fallbacks = nfb;
  return bad;
}

// Same step carrying one tangent direction (forward mode).
long orc_step_dual(const orc_params* P, const double* W, const double* dW, double* Wout,
                   double* dWout, double dt) {
  // forward-mode derivatives of TENO-D steps only (the comparison schemes'
  // nonlinear weights are evaluated on plain values)
  if (check_params(P) || !(dt > 0) || P->scheme != 0) return -1;
  const Grid g(*P);
  const size_t n = (size_t)g.nc * g.ncell;
  std::vector<Dual> a(n), b(n);
  for (size_t i = 0; i < n; ++i) a[i] = Dual(W[i], dW[i]);
  const long bad = s2o4_step<Dual>(*P, a.data(), b.data(), dt, nullptr, nullptr);
  for (size_t i = 0; i < n; ++i) {
    Wout[i] = b[i].v;
    dWout[i] = b[i].d;
  }
  return bad;
}

int orc_cfl_dt(const orc_params* P, const double* W, double cfl, double* dt) {
  if (check_params(P)) return -1;
  *dt = cfl_dt(*P, W, cfl);
  return 0;
}

// Advance W in place.  fixed_dt > 0: constant step; otherwise CFL steps,
// the last one clipped to t_end when t_end > 0.  Stops after max_steps steps
// or at t_end.  The time t runs from 0; the prescribed boundary states are
// those of time t0 + t.  Returns the number of failing Gauss-point
// evaluations.
long orc_run(const orc_params* P, double* W, int max_steps, double cfl, double t_end,
             double fixed_dt, double* t_out, int* steps_out, double t0) {
  if (check_params(P)) return -1;
  const Grid g(*P);
  std::vector<double> tmp((size_t)g.nc * g.ncell);
  double t = 0.0;
  int s = 0;
  long bad = 0;
  while (s < max_steps) {
    if (t_end > 0.0 && t >= t_end * (1.0 - 1e-14)) break;
    double dt = fixed_dt > 0.0 ? fixed_dt : cfl_dt(*P, W, cfl);
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    if (!(dt > 0.0)) return -2;
    bad += s2o4_step<double>(*P, W, tmp.data(), dt, nullptr, nullptr, t0 + t);
    std::copy(tmp.begin(), tmp.end(), W);
    t += dt;
    ++s;
  }
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = s;
  return bad;
}

}  // extern "C"
