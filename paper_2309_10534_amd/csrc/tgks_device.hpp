// tgks_device.hpp -- device math of the TENO-D gas-kinetic scheme (gfx950, FP64).
//
// Mu et al., "High-order gas-kinetic scheme with TENO class reconstruction for
// the Euler and Navier-Stokes equations", arXiv:2309.10534.
//
//   * TENO-D selection and candidate values (Sec. 4.2, Eqs. 4.5-4.14; the
//     candidate polynomials of Sec. 3.1-3.2, slopes Eqs. 3.22-3.24).
//   * Tangential Gauss-point reconstruction (Sec. 3.2 Steps 1-3).
//   * Gas-kinetic flux at one Gauss point (Sec. 2.1, Eqs. 2.2-2.9 with the
//     kinetic weighting of Eqs. 3.25-3.26), in closed form: Maxwellian moment
//     tables by the half-space erfc/exp recursion, closed-form solution of the
//     micro-slope systems, moment sums over psi.
//
// The selection arithmetic (smoothness indicators, gamma_k, cut-offs) and the
// candidate values follow one fixed evaluation order (constant divisors as
// multiplications by their correctly rounded reciprocals) with floating-point
// contraction disabled, so that the stencil flags are a deterministic
// function of the input bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// Every function is a template on the scalar type R: double in the kernels,
// an operation-counting type on the host (algorithmic flop counts).
#define TGKS_HD __host__ __device__ __forceinline__

namespace tgks {

// bits of TenoCfg::fast
constexpr int TENO_RATIO_OK = 1;   // the fixed ratios of teno_flag hold (teno_cfg)
constexpr int TENO_FILTER_OK = 2;  // the approximate-reciprocal test of teno_flag is valid

struct TenoCfg {
  double ct1, ct2, eps;
  int q;
  int fast;  // TENO_RATIO_OK | TENO_FILTER_OK where they hold (teno_cfg)
};

// The selection parameters, with the fast bits set where teno_flag's
// shortcuts are exact.
//
// TENO_RATIO_OK, fixed ratios of the certain decisions.  With b_k = beta_k
// + eps, gamma_k = b_k^-7 (q = 7) and m = min(b_0, b_1, b_2), whose gamma
// is the largest of the small stencils':
//   b_3 <= 4 m: gamma_3 / sum_{k<=3} gamma >= 1 / (3 4^7 + 1) (the three
//       small gammas at most gamma_max each): the large stencil is kept
//       (Eq. 4.7) if C_T1 <= 1 / (3 4^7 + 1) = 2.03e-5;
//   b_3 > 16 m: gamma_3 / sum < 1 / (16^7 + 1) (the sum holds gamma_max):
//       rejected if C_T1 >= 1 / (16^7 + 1) = 3.7e-9;
//   then b_k <= 4 m: gamma_k / sum_{k<3} gamma >= 1 / (2 4^7 + 1): kept
//       (Eq. 4.12) if C_T2 <= 3.05e-5; b_k > 8 m: gamma_k / sum <
//       1 / (8^7 + 1): dropped if C_T2 >= 4.8e-7.
// Each bound is reached in the limit (equal small indicators for the keeps,
// the other small stencils infinitely rough for the rejections).  The
// ratios are powers of two (exact products), and the cut-offs must clear
// each bound by a relative 1e-9, far above the rounding of the weights'
// evaluation (a few ulps of b^7, its reciprocal and the sums).  Also
// q = 7 and eps >= 1e-40 (b^7 and 1 / b^7 stay finite and normal).  The
// paper's C_T1 = 1e-7, C_T2 = 1e-5 are inside.
//
// TENO_FILTER_OK, the weights from approximate reciprocals with a margin
// (teno_flag): q = 7, eps >= 1e-40 and 1e-20 <= C_T1, C_T2 <= 1/2, so that
// every b^7, weight, sum and threshold of the test is a normal number
// (b in [eps, 1e40): b^7 and 1 / b^7 in [1e-280, 1e280]; a threshold
// C_T s >= 1e-20 1e-280 / 2, since the small weights hold at least half of
// the sum when the large stencil is rejected, C_T1 <= 1/2).
inline TenoCfg teno_cfg(double ct1, double ct2, double eps, int q) {
  const double d = 1e-9;
  const bool ok = q == 7 && eps >= 1e-40 && ct1 * (1.0 + d) <= 1.0 / (3.0 * 16384.0 + 1.0) &&
                  ct1 * (1.0 - d) >= 1.0 / (268435456.0 + 1.0) && ct2 * (1.0 + d) <= 1.0 / (2.0 * 16384.0 + 1.0) &&
                  ct2 * (1.0 - d) >= 1.0 / (2097152.0 + 1.0);
  const bool filt = q == 7 && eps >= 1e-40 && eps < 1e40 && ct1 >= 1e-20 && ct1 <= 0.5 && ct2 >= 1e-20 &&
                    ct2 <= 0.5;
  return TenoCfg{ct1, ct2, eps, q, (ok ? TENO_RATIO_OK : 0) | (filt ? TENO_FILTER_OK : 0)};
}

// An approximate reciprocal: the device's one-instruction estimate (its
// error is not assumed: teno_flag measures it by the residual 1 - x r).  On
// the host, 1 / x with the low 29 bits of the significand cleared (relative
// error up to 2^-23), so that host checks exercise the same error handling.
TGKS_HD double rcp_approx(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(x);
#else
  double r = 1.0 / x;
  uint64_t u;
  __builtin_memcpy(&u, &r, sizeof u);
  u &= ~((uint64_t(1) << 29) - 1);
  __builtin_memcpy(&r, &u, sizeof r);
  return r;
#endif
}

// 1/x to about one ulp (not always correctly rounded): the estimate and two
// Newton steps, each of which squares its relative error; for quantities
// that feed only the flux.  0 and infinities give NaN (the states they come
// from are rejected as non-physical).  The operation-counting type counts
// one division.
template <class R>
TGKS_HD R recip(R x) {
  return R(1.0) / x;
}
TGKS_HD double recip(double x) {
  double r = rcp_approx(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// ---------------------------------------------------------------------------
// TENO-D selection (Sec. 4.2).  q[0..4] = Q_{-2..2}.
// flag bit0 = delta_{3,1}; if it is 0, bits 1..3 = delta_{0,2}, delta_{1,2},
// delta_{2,2}.
//
// The flag is a function of the input bits: the weights gamma_k =
// (beta_k + eps)^-7 by correctly rounded divisions, summed and compared in
// one fixed order (SEL_EXACT).  The other modes reach the same flag, bit
// for bit, with less work where the decision is certain, and evaluate the
// weights exactly where it is not:
//
// SEL_FILTER: approximate reciprocals r_k of p_k = b_k^7 (one instruction
// each instead of a division) with their residuals e_k = 1 - p_k r_k (one
// fused multiply-add, rounded once).  If sum |e_k| <= 2^-18, each r_k is
// within a relative E = 2^-18 (1 + 2^-52) of 1/p_k, so within E + 2^-53
// of the correctly rounded weight g_k.  The sums of the positive r_k
// (two or three additions, same order) are then within E + 7 2^-53 of
// the exact path's sums, and the thresholds C_T s within E + 8 2^-53.  A
// comparison is certain when r_k clears the threshold by a factor
// 1 -+ 2^-12 (rounded once more): r_k > tau (1 + 2^-12) gives g_k > T and
// r_k < tau (1 - 2^-12) gives g_k < T, since 2^-12 exceeds twice E plus
// ten rounding errors 32-fold.  Undecided inputs (within 2.4e-4 of a
// cut-off, or a failed residual or range test) take the exact weights;
// on the benchmarks that is rare, so wavefronts seldom split.  All
// comparisons are evaluated (no short-circuit branches): one branch, to
// the exact weights, remains.
//
// SEL_RATIO: the fixed ratios of teno_cfg (when TENO_RATIO_OK; no
// reciprocal at all), then the exact weights.  Smooth data keeps the large
// stencil there; constant data (the quadratics' indicators vanish exactly,
// the quartic's keeps a rounding residue) rejects it there with all three
// quadratics kept.  The 3-D kernels use it (Taylor-Green vortex, smooth;
// 2.09 ms per face launch, against 2.12 with SEL_FILTER after the ratios
// and 2.28 with SEL_FILTER alone).  The 1-D and 2-D kernels use SEL_FILTER:
// on the four-quadrant Riemann problem most wavefronts mix lanes that the
// ratios decide and lanes they leave open after a few hundred steps (the
// ratios cost 4 % over 500 steps there, SEL_FILTER saves 3.5 %).
//
// A NaN or b >= 1e40 fails the range test (b_0 + .. + b_3 < 1e40) and
// takes the exact path.  The ratios and margins are literals so that they
// take no scalar registers (ratios held in the kernel arguments made the
// 2-D face kernel spill scalar registers into vector lanes).  The
// operation-counting type always evaluates the exact weights.
// ---------------------------------------------------------------------------
constexpr int SEL_EXACT = 0, SEL_FILTER = 1, SEL_RATIO = 2;

template <int MODE = SEL_EXACT, class R>
TGKS_HD unsigned teno_flag(const R* Q, const TenoCfg& c) {
#pragma clang fp contract(off)
  const R a = Q[0], b = Q[1], cc = Q[2], d = Q[3], e = Q[4];
  const double k13 = 13.0 / 12.0;
  R t1, t2, beta[4];
  t1 = (a - 2.0 * b) + cc;
  t2 = (a - 4.0 * b) + 3.0 * cc;
  beta[0] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (b - 2.0 * cc) + d;
  t2 = b - d;
  beta[1] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (cc - 2.0 * d) + e;
  t2 = (3.0 * cc - 4.0 * d) + e;
  beta[2] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  // quartic indicator (Eq. 3.7, q = 4) as a sum of squares of its derivatives
  const R P1 = (82.0 * (d - b) - 11.0 * (e - a)) * (1.0 / 120.0);
  const R P2 = ((((40.0 * b - 3.0 * a) - 74.0 * cc) + 40.0 * d) - 3.0 * e) * (1.0 / 56.0);
  const R P3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
  const R P4 = ((((a - 4.0 * b) + 6.0 * cc) - 4.0 * d) + e) * (1.0 / 24.0);
  const R s1 = P1 + P3 * (1.0 / 10.0);
  const R s2 = P2 + (123.0 / 455.0) * P4;
  beta[3] = (((s1 * s1) + (13.0 / 3.0) * (s2 * s2)) + (781.0 / 20.0) * (P3 * P3)) +
            (1421461.0 / 2275.0) * (P4 * P4);
  if constexpr (MODE == SEL_RATIO && std::is_same_v<R, double>) {
    if (c.fast & TENO_RATIO_OK) {
      const R b0 = beta[0] + c.eps, b1 = beta[1] + c.eps, b2 = beta[2] + c.eps, b3 = beta[3] + c.eps;
      if ((b0 + b1) + (b2 + b3) < 1e40) {
        const R m = fmin(fmin(b0, b1), b2);
        if (b3 <= 4.0 * m) return 1u;
        if (b3 > 16.0 * m) {
          const R lo = 4.0 * m, hi = 8.0 * m;
          const bool sure = !(b0 > lo && b0 <= hi) && !(b1 > lo && b1 <= hi) && !(b2 > lo && b2 <= hi);
          if (sure) return (b0 <= lo ? 2u : 0u) | (b1 <= lo ? 4u : 0u) | (b2 <= lo ? 8u : 0u);
        }
      }
    }
  }
  if constexpr (MODE == SEL_FILTER && std::is_same_v<R, double>) {
    if (c.fast & TENO_FILTER_OK) {
      const R b0 = beta[0] + c.eps, b1 = beta[1] + c.eps, b2 = beta[2] + c.eps, b3 = beta[3] + c.eps;
      const bool inr = (b0 + b1) + (b2 + b3) < 1e40;
      // every comparison evaluated, one branch to the exact weights
      R p[4], r[4], es = R(0.0);
      const R bb[4] = {b0, b1, b2, b3};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const R x2 = bb[k] * bb[k];
        const R x4 = x2 * x2;
        p[k] = (x4 * x2) * bb[k];
        r[k] = rcp_approx(p[k]);
        es += fabs(fma(-p[k], r[k], 1.0));
      }
      const R s3 = (r[0] + r[1]) + r[2];
      const R th1 = c.ct1 * (s3 + r[3]), th2 = c.ct2 * s3;
      const double up = 1.0 + 0x1p-12, dn = 1.0 - 0x1p-12;
      const R h2 = th2 * up, l2 = th2 * dn;
      const bool keep = r[3] > th1 * up, rej = r[3] < th1 * dn;
      const bool k0 = r[0] > h2, k1 = r[1] > h2, k2 = r[2] > h2;
      // (bitwise operators: no short-circuit branches)
      const bool sure = inr & (es <= 0x1p-18) &
                        (keep | (rej & (k0 | (r[0] < l2)) & (k1 | (r[1] < l2)) & (k2 | (r[2] < l2))));
      if (sure) return keep ? 1u : ((k0 ? 2u : 0u) | (k1 ? 4u : 0u) | (k2 ? 8u : 0u));
    }
  }
  R g[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const R bb = beta[k] + c.eps;
    R pw;
    if (c.q == 7) {
      const R b2 = bb * bb;
      const R b4 = b2 * b2;
      pw = (b4 * b2) * bb;
    } else {
      pw = R(1.0);
      for (int r = 0; r < c.q; ++r) pw = pw * bb;
    }
    g[k] = 1.0 / pw;  // gamma_k = (beta_k + eps)^-q  (Eq. 4.5)
  }
  const R s4 = ((g[0] + g[1]) + g[2]) + g[3];
  if (!(g[3] < c.ct1 * s4)) return 1u;  // large stencil kept (Eqs. 4.6-4.7)
  const R s3 = (g[0] + g[1]) + g[2];
  unsigned f = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!(g[k] < c.ct2 * s3)) f |= 2u << k;  // Eqs. 4.11-4.12
  return f;
}

// Values and slopes (cell units) at x_{i-1/2} and x_{i+1/2} of the selected
// reconstruction: out = {v(-1/2), s(-1/2), v(+1/2), s(+1/2)}.
template <class R>
TGKS_HD void teno_face(const R* Q, unsigned flag, R* out) {
#pragma clang fp contract(off)
  const R a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  if (flag & 1u) {
    // Eq. 4.8, Eq. 4.9 and their mirror images
    out[2] = ((((2.0 * a - 13.0 * b) + 47.0 * c) + 27.0 * d) - 3.0 * e) * (1.0 / 60.0);
    out[3] = (((b - 15.0 * c) + 15.0 * d) - e) * (1.0 / 12.0);
    out[0] = ((((27.0 * b - 3.0 * a) + 47.0 * c) - 13.0 * d) + 2.0 * e) * (1.0 / 60.0);
    out[1] = (((a - 15.0 * b) + 15.0 * c) - d) * (1.0 / 12.0);
    return;
  }
  // surviving small stencils averaged with d_k = 1/3 (Eqs. 4.13-4.14)
  // omega_k = d_k delta_k / sum d_k delta_k with d_k = 1/3: in double
  // arithmetic (1/3)/(m/3) is exactly 1, 0.5 or (1/3) for m = 1, 2, 3
  // surviving stencils
  const int cnt = (int)((flag >> 1) & 1u) + (int)((flag >> 2) & 1u) + (int)((flag >> 3) & 1u);
  const double om = cnt == 1 ? 1.0 : (cnt == 2 ? 0.5 : 1.0 / 3.0);
  const R o0 = R((flag & 2u) ? om : 0.0), o1 = R((flag & 4u) ? om : 0.0), o2 = R((flag & 8u) ? om : 0.0);
  const R vp0 = ((2.0 * a - 7.0 * b) + 11.0 * c) * (1.0 / 6.0);
  const R vp1 = ((5.0 * c - b) + 2.0 * d) * (1.0 / 6.0);
  const R vp2 = ((2.0 * c + 5.0 * d) - e) * (1.0 / 6.0);
  const R dp0 = (a - 3.0 * b) + 2.0 * c;
  const R dp12 = d - c;
  const R vm0 = ((5.0 * b - a) + 2.0 * c) * (1.0 / 6.0);
  const R vm1 = ((2.0 * b + 5.0 * c) - d) * (1.0 / 6.0);
  const R vm2 = ((11.0 * c - 7.0 * d) + 2.0 * e) * (1.0 / 6.0);
  const R dm01 = c - b;
  const R dm2 = (3.0 * d - 2.0 * c) - e;
  const R z = R(0.0);
  out[0] = ((z + o0 * vm0) + o1 * vm1) + o2 * vm2;
  out[1] = ((z + o0 * dm01) + o1 * dm01) + o2 * dm2;
  out[2] = ((z + o0 * vp0) + o1 * vp1) + o2 * vp2;
  out[3] = ((z + o0 * dp0) + o1 * dp12) + o2 * dp12;
}

// Selected polynomial at the Gauss points s = -+1/(2 sqrt 3) (cell units):
// val[m], der[m] for m = 0 (s-) and 1 (s+).  The values feed only the flux,
// so contraction is allowed here.
template <class R>
TGKS_HD void teno_gauss(const R* Q, unsigned flag, R* val, R* der) {
  const R a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  const double s = 0.28867513459481288225;  // 1/(2 sqrt 3)
  R c0, c1, c2, c3 = R(0.0), c4 = R(0.0);
  if (flag & 1u) {
    c0 = ((2134.0 * c - 116.0 * (d + b)) + 9.0 * (e + a)) * (1.0 / 1920.0);
    c1 = (34.0 * (d - b) - 5.0 * (e - a)) * (1.0 / 48.0);
    c2 = ((12.0 * (d + b) - 22.0 * c) - (e + a)) * (1.0 / 16.0);
    c3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
    c4 = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) * (1.0 / 24.0);
  } else {
    const bool k0 = flag & 2u, k1 = flag & 4u, k2 = flag & 8u;
    const int cnt = (int)k0 + (int)k1 + (int)k2;
    const double inv = cnt == 1 ? 1.0 : (cnt == 2 ? 0.5 : 1.0 / 3.0);
    R s0 = R(0.0), s1 = R(0.0), s2 = R(0.0);
    if (k0) {
      s0 += (23.0 * c + 2.0 * b - a) * (1.0 / 24.0);
      s1 += (3.0 * c - 4.0 * b + a) * 0.5;
      s2 += (c - 2.0 * b + a) * 0.5;
    }
    if (k1) {
      s0 += (26.0 * c - d - b) * (1.0 / 24.0);
      s1 += (d - b) * 0.5;
      s2 += (d + b - 2.0 * c) * 0.5;
    }
    if (k2) {
      s0 += (23.0 * c + 2.0 * d - e) * (1.0 / 24.0);
      s1 += (4.0 * d - 3.0 * c - e) * 0.5;
      s2 += (c - 2.0 * d + e) * 0.5;
    }
    c0 = s0 * inv;
    c1 = s1 * inv;
    c2 = s2 * inv;
  }
  const double ss = s * s;
  const R even = c0 + ss * (c2 + ss * c4);  // even part of p at +-s
  const R odd = s * (c1 + ss * c3);
  val[0] = even - odd;
  val[1] = even + odd;
  const R deven = c1 + (3.0 * ss) * c3;  // even part of p' at +-s
  const R dodd = s * (2.0 * c2 + (4.0 * ss) * c4);
  der[0] = deven - dodd;
  der[1] = deven + dodd;
}

// teno_gauss in one fixed evaluation order without contraction: the 3-D
// first sweep's Gauss-point values are the inputs of the second sweep's
// selections, whose flags must be a deterministic function of the data.
template <class R>
TGKS_HD void teno_gauss_exact(const R* Q, unsigned flag, R* val, R* der) {
#pragma clang fp contract(off)
  const R a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  const double s = 0.28867513459481288225;  // 1/(2 sqrt 3)
  R c0, c1, c2, c3 = R(0.0), c4 = R(0.0);
  if (flag & 1u) {
    c0 = ((2134.0 * c - 116.0 * (d + b)) + 9.0 * (e + a)) * (1.0 / 1920.0);
    c1 = (34.0 * (d - b) - 5.0 * (e - a)) * (1.0 / 48.0);
    c2 = ((12.0 * (d + b) - 22.0 * c) - (e + a)) * (1.0 / 16.0);
    c3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
    c4 = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) * (1.0 / 24.0);
  } else {
    const bool k0 = flag & 2u, k1 = flag & 4u, k2 = flag & 8u;
    const int cnt = (int)k0 + (int)k1 + (int)k2;
    const double inv = cnt == 1 ? 1.0 : (cnt == 2 ? 0.5 : 1.0 / 3.0);
    R s0 = R(0.0), s1 = R(0.0), s2 = R(0.0);
    if (k0) {
      s0 = s0 + ((23.0 * c + 2.0 * b) - a) * (1.0 / 24.0);
      s1 = s1 + ((3.0 * c - 4.0 * b) + a) * 0.5;
      s2 = s2 + ((c - 2.0 * b) + a) * 0.5;
    }
    if (k1) {
      s0 = s0 + ((26.0 * c - d) - b) * (1.0 / 24.0);
      s1 = s1 + (d - b) * 0.5;
      s2 = s2 + ((d + b) - 2.0 * c) * 0.5;
    }
    if (k2) {
      s0 = s0 + ((23.0 * c + 2.0 * d) - e) * (1.0 / 24.0);
      s1 = s1 + ((4.0 * d - 3.0 * c) - e) * 0.5;
      s2 = s2 + ((c - 2.0 * d) + e) * 0.5;
    }
    c0 = s0 * inv;
    c1 = s1 * inv;
    c2 = s2 * inv;
  }
  const double ss = s * s;
  const R even = c0 + ss * (c2 + ss * c4);
  const R odd = s * (c1 + ss * c3);
  val[0] = even - odd;
  val[1] = even + odd;
  const R deven = c1 + (3.0 * ss) * c3;
  const R dodd = s * (2.0 * c2 + (4.0 * ss) * c4);
  der[0] = deven - dodd;
  der[1] = deven + dodd;
}

// The selected polynomial at one Gauss point m (0: s-, 1: s+), cell units.
template <class R>
TGKS_HD void teno_gauss_at(const R* Q, unsigned flag, int m, R& val, R& der) {
  R v[2], d[2];
  teno_gauss(Q, flag, v, d);
  val = m ? v[1] : v[0];
  der = m ? d[1] : d[0];
}

// ---------------------------------------------------------------------------
// The paper's comparison schemes on the same five values and candidate
// polynomials: WENO-AO (Sec. 3.2), TENO5 (Sec. 4.1) and WENO-Z (Sec. 3.1).
//   * WENO-AO: linear weights d3 = d_Hi, d0 = d2 = (1 - d_Hi)(1 - d_Lo)/2,
//     d1 = (1 - d_Hi) d_Lo; omega_k = d_k (1 + (tau / (beta_k + eps))^2)
//     with tau the mean of |beta3 - beta_k| (the ratio squared, as Table 2
//     requires), normalised over k = 0..3; the polynomial
//     w3 (p3/d3 - sum d_k/d3 p_k) + sum w_k p_k gives values and slopes
//     wherever they are needed (interfaces, Gauss points).
//   * WENO-Z / TENO5: small stencils only, omega_k = d_k (1 + tau /
//     (beta_k + eps)) (WENO-Z) or d_k delta_k with delta_k = 0 where
//     (1 + tau / (beta_k + eps))^q < C_T sum (TENO5), tau = |beta0 - beta2|,
//     d_k the linear weights of the evaluation point (0.1, 0.6, 0.3 at
//     x_{i+1/2}, mirrored at x_{i-1/2}, (7/36 -+ sqrt 3/1080, 11/18, ...) at
//     the Gauss points).  Interface slopes from the quadratic with the cell
//     average and the two interface values (Eq. 3.11); along a face the
//     same quadratic's derivative at the Gauss point.
// The TENO5 cut-offs and the WENO-Z / TENO5 interface values follow one
// fixed evaluation order without contraction (the interface values are the
// inputs of the tangential selections, whose flags must be a deterministic
// function of the data).
// ---------------------------------------------------------------------------
constexpr int SCHEME_TENO_D = 0, SCHEME_WENO_AO = 1, SCHEME_TENO5 = 2, SCHEME_WENO_Z = 3;

struct SchemeCfg {
  double ct, eps;      // TENO5 cut-off C_T and epsilon
  int q;               // TENO5 power
  double d_hi, d_lo;   // WENO-AO linear weights
  double eps_w;        // WENO-AO / WENO-Z epsilon
};

// Jiang-Shu indicators of p0..p2 and Balsara's form for p3 (the same
// arithmetic as teno_flag's)
template <class R>
TGKS_HD void indicators(const R* Q, R* beta) {
#pragma clang fp contract(off)
  const R a = Q[0], b = Q[1], cc = Q[2], d = Q[3], e = Q[4];
  const double k13 = 13.0 / 12.0;
  R t1, t2;
  t1 = (a - 2.0 * b) + cc;
  t2 = (a - 4.0 * b) + 3.0 * cc;
  beta[0] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (b - 2.0 * cc) + d;
  t2 = b - d;
  beta[1] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  t1 = (cc - 2.0 * d) + e;
  t2 = (3.0 * cc - 4.0 * d) + e;
  beta[2] = k13 * (t1 * t1) + 0.25 * (t2 * t2);
  const R P1 = (82.0 * (d - b) - 11.0 * (e - a)) * (1.0 / 120.0);
  const R P2 = ((((40.0 * b - 3.0 * a) - 74.0 * cc) + 40.0 * d) - 3.0 * e) * (1.0 / 56.0);
  const R P3 = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
  const R P4 = ((((a - 4.0 * b) + 6.0 * cc) - 4.0 * d) + e) * (1.0 / 24.0);
  const R s1 = P1 + P3 * (1.0 / 10.0);
  const R s2 = P2 + (123.0 / 455.0) * P4;
  beta[3] = (((s1 * s1) + (13.0 / 3.0) * (s2 * s2)) + (781.0 / 20.0) * (P3 * P3)) +
            (1421461.0 / 2275.0) * (P4 * P4);
}

// TENO5 cut-offs: bit k = delta_k (Eqs. 4.1-4.3)
template <class R>
TGKS_HD unsigned teno5_flags(const R* beta, const SchemeCfg& c) {
#pragma clang fp contract(off)
  const R tau = fabs(beta[0] - beta[2]);
  R g[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const R t = 1.0 + tau / (beta[k] + c.eps);
    R pw;
    if (c.q == 6) {
      const R t2 = t * t;
      const R t4 = t2 * t2;
      pw = t4 * t2;
    } else {
      pw = R(1.0);
      for (int r = 0; r < c.q; ++r) pw = pw * t;
    }
    g[k] = pw;
  }
  const R sg = (g[0] + g[1]) + g[2];
  unsigned f = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!(g[k] < c.ct * sg)) f |= 1u << k;
  return f;
}

// linear weights of p0..p2 at x_{i-1/2} (where 0), x_{i+1/2} (1), the Gauss
// points -1/(2 sqrt 3) (2) and +1/(2 sqrt 3) (3)
TGKS_HD void lin_weights(int where, double* d) {
  const double gw = 1.7320508075688772 / 1080.0;
  if (where == 0) {
    d[0] = 0.3; d[1] = 0.6; d[2] = 0.1;
  } else if (where == 1) {
    d[0] = 0.1; d[1] = 0.6; d[2] = 0.3;
  } else if (where == 2) {
    d[0] = 7.0 / 36.0 + gw; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 - gw;
  } else {
    d[0] = 7.0 / 36.0 - gw; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 + gw;
  }
}

// normalised weights of p0..p2 at point `where`: TENO5 from its flags,
// WENO-Z from the indicators
template <int SCHEME, class R>
TGKS_HD void small_weights(const R* beta, unsigned flag, int where, const SchemeCfg& c, R* ob) {
#pragma clang fp contract(off)
  double d[3];
  lin_weights(where, d);
  if (SCHEME == SCHEME_TENO5) {
    double S = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) S = S + ((flag >> k) & 1u ? d[k] : 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) ob[k] = R((flag >> k) & 1u ? d[k] / S : 0.0);
  } else {
    const R tau = fabs(beta[0] - beta[2]);
    R om[3], S = R(0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      om[k] = d[k] * (1.0 + tau / (beta[k] + c.eps_w));
      S = S + om[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ob[k] = om[k] / S;
  }
}

// WENO-AO coefficients of p0..p2 (w[0..2]) and p3 (w[3])
template <class R>
TGKS_HD void ao_coeffs(const R* beta, const SchemeCfg& c, R* w) {
  const double dh = c.d_hi, dl = c.d_lo;
  const double d[4] = {(1.0 - dh) * (1.0 - dl) / 2.0, (1.0 - dh) * dl, (1.0 - dh) * (1.0 - dl) / 2.0, dh};
  const R tau = ((fabs(beta[3] - beta[0]) + fabs(beta[3] - beta[1])) + fabs(beta[3] - beta[2])) * (1.0 / 3.0);
  R om[4], S = R(0.0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const R r = tau / (beta[k] + c.eps_w);
    om[k] = d[k] * (1.0 + r * r);
    S = S + om[k];
  }
  const R iS = R(1.0) / S;
  const R o3 = om[3] * iS;
  w[3] = o3 * (1.0 / dh);
#pragma unroll
  for (int k = 0; k < 3; ++k) w[k] = om[k] * iS - o3 * (d[k] / dh);
}

// interface values of p0..p2 at x_{i-1/2} (vm) and x_{i+1/2} (vp)
template <class R>
TGKS_HD void small_face(const R* Q, R* vm, R* vp) {
#pragma clang fp contract(off)
  const R a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  vp[0] = ((2.0 * a - 7.0 * b) + 11.0 * c) * (1.0 / 6.0);
  vp[1] = ((5.0 * c - b) + 2.0 * d) * (1.0 / 6.0);
  vp[2] = ((2.0 * c + 5.0 * d) - e) * (1.0 / 6.0);
  vm[0] = ((5.0 * b - a) + 2.0 * c) * (1.0 / 6.0);
  vm[1] = ((2.0 * b + 5.0 * c) - d) * (1.0 / 6.0);
  vm[2] = ((11.0 * c - 7.0 * d) + 2.0 * e) * (1.0 / 6.0);
}

// WENO-Z / TENO5 interface values v(-1/2), v(+1/2); returns the flags
template <int SCHEME, class R>
TGKS_HD unsigned zt_face(const R* Q, const R* beta, const SchemeCfg& c, R& vm_o, R& vp_o) {
#pragma clang fp contract(off)
  const unsigned f = SCHEME == SCHEME_TENO5 ? teno5_flags(beta, c) : 0u;
  R om[3], op[3], vm[3], vp[3];
  small_weights<SCHEME>(beta, f, 0, c, om);
  small_weights<SCHEME>(beta, f, 1, c, op);
  small_face(Q, vm, vp);
  R a = R(0.0), b = R(0.0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a = a + om[k] * vm[k];
    b = b + op[k] * vp[k];
  }
  vm_o = a;
  vp_o = b;
  return f;
}

// Normal reconstruction: out = {v(-1/2), s(-1/2), v(+1/2), s(+1/2)} (cell
// units); returns the flags (TENO5) or 0
template <int SCHEME, class R>
TGKS_HD unsigned scheme_face(const R* Q, const SchemeCfg& c, R* out) {
#pragma clang fp contract(off)
  R beta[4];
  indicators(Q, beta);
  if (SCHEME == SCHEME_WENO_AO) {
    R w[4];
    ao_coeffs(beta, c, w);
    const R a = Q[0], b = Q[1], cc = Q[2], d = Q[3], e = Q[4];
    R vm[3], vp[3];
    small_face(Q, vm, vp);
    const R Lp = ((((2.0 * a - 13.0 * b) + 47.0 * cc) + 27.0 * d) - 3.0 * e) * (1.0 / 60.0);
    const R Lps = (((b - 15.0 * cc) + 15.0 * d) - e) * (1.0 / 12.0);
    const R Lm = ((((27.0 * b - 3.0 * a) + 47.0 * cc) - 13.0 * d) + 2.0 * e) * (1.0 / 60.0);
    const R Lms = (((a - 15.0 * b) + 15.0 * cc) - d) * (1.0 / 12.0);
    const R dp0 = (a - 3.0 * b) + 2.0 * cc, dp12 = d - cc;
    const R dm01 = cc - b, dm2 = (3.0 * d - 2.0 * cc) - e;
    out[0] = ((w[3] * Lm + w[0] * vm[0]) + w[1] * vm[1]) + w[2] * vm[2];
    out[1] = ((w[3] * Lms + w[0] * dm01) + w[1] * dm01) + w[2] * dm2;
    out[2] = ((w[3] * Lp + w[0] * vp[0]) + w[1] * vp[1]) + w[2] * vp[2];
    out[3] = ((w[3] * Lps + w[0] * dp0) + w[1] * dp12) + w[2] * dp12;
    return 0u;
  }
  R vm, vp;
  const unsigned f = zt_face<SCHEME>(Q, beta, c, vm, vp);
  out[0] = vm;
  out[1] = -2.0 * ((2.0 * vm + vp) - 3.0 * Q[2]);
  out[2] = vp;
  out[3] = 2.0 * ((vm + 2.0 * vp) - 3.0 * Q[2]);
  return f;
}

// monomial coefficients (x in [-1/2, 1/2]) of the large-stencil quartic (L)
// and the three quadratics (S[k][0..2])
template <class R>
TGKS_HD void cand_coeffs(const R* Q, R* L, R (*S)[3]) {
  const R a = Q[0], b = Q[1], c = Q[2], d = Q[3], e = Q[4];
  L[0] = ((2134.0 * c - 116.0 * (d + b)) + 9.0 * (e + a)) * (1.0 / 1920.0);
  L[1] = (34.0 * (d - b) - 5.0 * (e - a)) * (1.0 / 48.0);
  L[2] = ((12.0 * (d + b) - 22.0 * c) - (e + a)) * (1.0 / 16.0);
  L[3] = ((e - a) - 2.0 * (d - b)) * (1.0 / 12.0);
  L[4] = ((((a - 4.0 * b) + 6.0 * c) - 4.0 * d) + e) * (1.0 / 24.0);
  S[0][0] = (23.0 * c + 2.0 * b - a) * (1.0 / 24.0);
  S[0][1] = (3.0 * c - 4.0 * b + a) * 0.5;
  S[0][2] = (c - 2.0 * b + a) * 0.5;
  S[1][0] = (26.0 * c - d - b) * (1.0 / 24.0);
  S[1][1] = (d - b) * 0.5;
  S[1][2] = (d + b - 2.0 * c) * 0.5;
  S[2][0] = (23.0 * c + 2.0 * d - e) * (1.0 / 24.0);
  S[2][1] = (4.0 * d - 3.0 * c - e) * 0.5;
  S[2][2] = (c - 2.0 * d + e) * 0.5;
}

// Tangential reconstruction at the Gauss points s = -+1/(2 sqrt 3): val[m],
// der[m] (cell units); returns the flags (TENO5) or 0
template <int SCHEME, class R>
TGKS_HD unsigned scheme_gauss(const R* Q, const SchemeCfg& c, R* val, R* der) {
  const double s = 0.28867513459481288225;  // 1/(2 sqrt 3)
  const double ss = s * s;
  R beta[4], L[5], S[3][3];
  indicators(Q, beta);
  cand_coeffs(Q, L, S);
  if (SCHEME == SCHEME_WENO_AO) {
    R w[4];
    ao_coeffs(beta, c, w);
    const R c0 = w[3] * L[0] + ((w[0] * S[0][0] + w[1] * S[1][0]) + w[2] * S[2][0]);
    const R c1 = w[3] * L[1] + ((w[0] * S[0][1] + w[1] * S[1][1]) + w[2] * S[2][1]);
    const R c2 = w[3] * L[2] + ((w[0] * S[0][2] + w[1] * S[1][2]) + w[2] * S[2][2]);
    const R c3 = w[3] * L[3], c4 = w[3] * L[4];
    const R even = c0 + ss * (c2 + ss * c4), odd = s * (c1 + ss * c3);
    val[0] = even - odd;
    val[1] = even + odd;
    const R deven = c1 + (3.0 * ss) * c3, dodd = s * (2.0 * c2 + (4.0 * ss) * c4);
    der[0] = deven - dodd;
    der[1] = deven + dodd;
    return 0u;
  }
  R vm, vp;
  const unsigned f = zt_face<SCHEME>(Q, beta, c, vm, vp);
  // slopes: the quadratic with the average Q_0 and the end values vm, vp
  const R q1 = vp - vm, q2 = 3.0 * (vm + vp) - 6.0 * Q[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    R ob[3];
    small_weights<SCHEME>(beta, f, 2 + m, c, ob);
    const R c0 = (ob[0] * S[0][0] + ob[1] * S[1][0]) + ob[2] * S[2][0];
    const R c1 = (ob[0] * S[0][1] + ob[1] * S[1][1]) + ob[2] * S[2][1];
    const R c2 = (ob[0] * S[0][2] + ob[1] * S[1][2]) + ob[2] * S[2][2];
    const double x = m ? s : -s;
    val[m] = c0 + x * (c1 + x * c2);
    der[m] = q1 + (2.0 * x) * q2;
  }
  return f;
}

// Eq. 3.12: the equilibrium slope at x_{i+1/2} from the cells i-1 .. i+2
// (cell units)
template <class R>
TGKS_HD R eq_slope(R wm1, R w0, R w1, R w2) {
  return (-1.0 / 12.0) * (w2 - wm1) + 1.25 * (w1 - w0);
}

// ---------------------------------------------------------------------------
// Characteristic variables: an optional choice of reconstruction variables
// (the paper reconstructs the conservative ones).  At a face the reference
// state Wb is the mean of the conservative states of the two adjacent cells
// (frame order: rho, m_0..m_{D-1}, E); the fields are the eigenvectors of the
// Euler flux Jacobian along frame axis A at Wb (A = 0 normal, A = 1 along
// the face), ordered u_A - c, entropy, shear waves of the other axes in
// increasing order, u_A + c.  L holds the left eigenvectors as rows, Rm the
// right ones as columns (Rm L = I).  Entries, projections and
// back-projections follow one fixed operation order without contraction
// (dense left-to-right sums over all components), so that the projected
// values, and the stencil selections made on them, are a deterministic
// function of the input bits.  A non-physical Wb gives the identity.
// ---------------------------------------------------------------------------
template <int D, int A, class R>
TGKS_HD bool char_basis(double gamma, const R* Wb, R (*L)[D + 2], R (*Rm)[D + 2]) {
#pragma clang fp contract(off)
  constexpr int NC = D + 2, KP = D + 1;
  const R rho = Wb[0];
  const R irho = R(1.0) / rho;
  R u[D];
#pragma unroll
  for (int e = 0; e < D; ++e) u[e] = Wb[1 + e] * irho;
  R q2 = u[0] * u[0];
#pragma unroll
  for (int e = 1; e < D; ++e) q2 = q2 + u[e] * u[e];
  const R E = Wb[D + 1];
  const R p = (gamma - 1.0) * (E - 0.5 * (rho * q2));
  const R c2 = (gamma * p) * irho;
  const bool ok = (rho > 0.0) && (p > 0.0) && (c2 < INFINITY) && (E < INFINITY) && (E > -INFINITY);
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) L[i][j] = Rm[i][j] = R(0.0);
  if (!ok) {
#pragma unroll
    for (int i = 0; i < NC; ++i) L[i][i] = Rm[i][i] = R(1.0);
    return false;
  }
  const R c = sqrt(c2);
  const R ic = R(1.0) / c;
  const R H = (E + p) * irho;
  const R b1 = (gamma - 1.0) / c2;
  const R b2 = 0.5 * (b1 * q2);
  const R un = u[A];
  const R uc = un * c;
  L[0][0] = 0.5 * (b2 + un * ic);
  L[KP][0] = 0.5 * (b2 - un * ic);
  L[1][0] = 1.0 - b2;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    if (e == A) {
      L[0][1 + e] = 0.5 * (-(b1 * un) - ic);
      L[KP][1 + e] = 0.5 * (ic - b1 * un);
    } else {
      L[0][1 + e] = 0.5 * (-(b1 * u[e]));
      L[KP][1 + e] = 0.5 * (-(b1 * u[e]));
    }
    L[1][1 + e] = b1 * u[e];
  }
  L[0][D + 1] = 0.5 * b1;
  L[KP][D + 1] = 0.5 * b1;
  L[1][D + 1] = -b1;
  int k = 2;
#pragma unroll
  for (int s = 0; s < D; ++s) {
    if (s == A) continue;
    L[k][0] = -u[s];
    L[k][1 + s] = R(1.0);
    Rm[1 + s][k] = R(1.0);
    Rm[D + 1][k] = u[s];
    ++k;
  }
  Rm[0][0] = R(1.0);
  Rm[0][1] = R(1.0);
  Rm[0][KP] = R(1.0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    Rm[1 + e][0] = e == A ? un - c : u[e];
    Rm[1 + e][1] = u[e];
    Rm[1 + e][KP] = e == A ? un + c : u[e];
  }
  Rm[D + 1][0] = H - uc;
  Rm[D + 1][1] = 0.5 * q2;
  Rm[D + 1][KP] = H + uc;
  return true;
}

// y = M x with dense left-to-right sums, no contraction
template <int NC, class R>
TGKS_HD void char_mv(const R (*M)[NC], const R* x, R* y) {
#pragma clang fp contract(off)
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    R v = M[i][0] * x[0];
#pragma unroll
    for (int j = 1; j < NC; ++j) v = v + M[i][j] * x[j];
    y[i] = v;
  }
}

// one row: l . x
template <int NC, class R>
TGKS_HD R char_dot(const R* l, const R* x) {
#pragma clang fp contract(off)
  R v = l[0] * x[0];
#pragma unroll
  for (int j = 1; j < NC; ++j) v = v + l[j] * x[j];
  return v;
}

// Normal reconstruction of both sides of one face in characteristic
// variables, from the six frame-ordered cells C[0..5] = f-3 .. f+2 along the
// normal: values and slopes (slopes per unit length, idn = 1/dx) in frame
// order; fr = selection flags of the right side (cell f at its low face).
template <int D, class R>
TGKS_HD void char_recon_face(double gamma, const R (*C)[D + 2], const TenoCfg& tn, double idn, R* vl, R* sl,
                             R* vr, R* sr, unsigned* fr) {
  constexpr int NC = D + 2;
  R Wb[NC], L[NC][NC], Rm[NC][NC];
  {
#pragma clang fp contract(off)
#pragma unroll
    for (int q = 0; q < NC; ++q) Wb[q] = 0.5 * (C[2][q] + C[3][q]);
  }
  char_basis<D, 0>(gamma, Wb, L, Rm);
  R ol[NC][4], orr[NC][4];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    R V[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) V[r] = char_dot<NC>(L[k], C[r]);
    const unsigned f0 = teno_flag<SEL_FILTER>(V, tn);
    const unsigned f1 = teno_flag<SEL_FILTER>(V + 1, tn);
    teno_face(V, f0, ol[k]);
    teno_face(V + 1, f1, orr[k]);
    fr[k] = f1;
  }
  R a[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) a[k] = ol[k][2];
  char_mv<NC>(Rm, a, vl);
#pragma unroll
  for (int k = 0; k < NC; ++k) a[k] = ol[k][3];
  char_mv<NC>(Rm, a, sl);
#pragma unroll
  for (int k = 0; k < NC; ++k) a[k] = orr[k][0];
  char_mv<NC>(Rm, a, vr);
#pragma unroll
  for (int k = 0; k < NC; ++k) a[k] = orr[k][1];
  char_mv<NC>(Rm, a, sr);
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    sl[q] = sl[q] * idn;
    sr[q] = sr[q] * idn;
  }
}

// ---------------------------------------------------------------------------
// Gas-kinetic flux at one Gauss point (Sec. 2.1), face frame: u1 is normal.
// ---------------------------------------------------------------------------
struct FluxCfg {
  double N;          // K + D = 2/(gamma - 1)
  double K;          // internal degrees of freedom
  double mu, pr_fix; // viscosity; (1/Pr - 1) for the energy flux, 0 if Euler
  double c1, c2;
  int tau_mode;      // 0 inviscid, 1 viscous, 2 zero
};

constexpr int NM1 = 7;  // normal moment table <u1^n>, n = 0..6
constexpr int NMT = 6;  // tangential tables <u_t^n>, n = 0..5

template <int D, class R>
struct Gas {
  R rho, irho, U[D], lam, h;  // h = 1/(2 lambda) = p / rho
  bool ok;
};

// 1/sqrt(x): the device's reciprocal square root in the kernels
template <class R>
TGKS_HD R rsqrt_(R x) {
  return rsqrt(x);
}
TGKS_HD double rsqrt_(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return rsqrt(x);
#else
  return 1.0 / sqrt(x);
#endif
}

// An opaque copy: the compiler cannot see that the result equals the input,
// so a recomputation from it is not merged with an earlier identical one
// (whose results would otherwise stay live in registers until the later
// use).  The value is unchanged.
template <class R>
TGKS_HD R opaque(R x) {
  return x;
}
TGKS_HD double opaque(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}

// (rho, 1/rho, U, lambda, h) of W with one reciprocal:
// re = rho (rho E) - |rho U|^2 / 2 = rho^2 e_int, inv = 1 / (rho re)
template <int D, class R>
TGKS_HD void make_gas(const R* W, double N, Gas<D, R>& g) {
  g.rho = W[0];
  R m2 = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) m2 += W[d + 1] * W[d + 1];
  const R re = g.rho * W[D + 1] - 0.5 * m2;
  const R inv = recip(g.rho * re);
  g.irho = re * inv;
#pragma unroll
  for (int d = 0; d < D; ++d) g.U[d] = W[d + 1] * g.irho;
  const R ir2 = g.irho * g.irho;
  g.h = ((2.0 / N) * re) * ir2;                      // p / rho = 1/(2 lambda)
  g.lam = (0.25 * N) * ((g.rho * g.rho) * (g.rho * inv));
  g.ok = (g.rho > 0.0) && (re > 0.0) && (g.rho < INFINITY) && (re < INFINITY);
}

template <class R>
TGKS_HD void full_table(R U, R h, R* m, int n) {
  m[0] = R(1.0);
  m[1] = U;
  for (int k = 1; k + 1 < n; ++k) m[k + 1] = U * m[k] + ((double)k * h) * m[k - 1];
}

// half-space table from its first two entries
template <class R>
TGKS_HD void half_table(R U, R h, R m0, R m1, R* m) {
  m[0] = m0;
  m[1] = m1;
#pragma unroll
  for (int k = 1; k + 1 < NM1; ++k) m[k + 1] = U * m[k] + ((double)k * h) * m[k - 1];
}

// erfc(x) given ex2 = exp(-x^2), which the half-space moments need anyway.
// With t = |x|: erfc(t) = ex2 f(y) / (1 + 2t), where f(y) = (1 + 2t)
// exp(t^2) erfc(t) is a smooth function of y = (t - K) / (t + K) on
// [-1, 1] (K = 3.75; the form of Shepherd and Laframboise, Math. Comp. 36,
// 1981): its Chebyshev series cut after 23 terms, in powers of y, summed by
// Horner's rule as even and odd parts in y^2 (two independent chains); the
// power coefficients are small (sum of magnitudes 1.76), so the power form
// is as accurate as the series.  erfc(-t) = 2 - erfc(t).  The
// coefficients are written by paper_2309_10534_amd/erfc_coeffs.py from the
// definition (mpmath, 40 digits); in this arithmetic f / (1 + 2t) is
// within 5.6e-16 of exp(t^2) erfc(t) for t in [0, 27] (beyond, ex2
// underflows).  One reciprocal of (t + K)(1 + 2t) (estimate and two Newton
// steps, about 1 ulp) serves both divisions.  The operation-counting type
// counts one erfc.
constexpr double ERFC_POLY[23] = {
    1.2375126308378275, -0.14024059858554525, 0.0035854154854790257,
    0.08227673848999506, -0.10880393014244462, 0.09230432116428125,
    -0.05869339857664934, 0.028362277372111139, -0.0097465796832652621,
    0.0017556261651970652, 0.00029371437804495801, -0.00029015535246077655,
    5.1646529741774162e-05, 2.2387565714911816e-05, -1.1438048033346894e-05,
    -9.7926257073035231e-07, 1.7419821586224816e-06, -5.0844653786873023e-08,
    -2.4857126248016745e-07, 1.8790823223700481e-08, 3.1979266716668042e-08,
    -1.9551358868985616e-09, -2.6231073471334759e-09,
};

template <class R>
TGKS_HD R erfc_exp(R x, R ex2) {
  return erfc(x);
}
TGKS_HD double erfc_exp(double x, double ex2) {
  const double K = 3.75;
  const double t = fmin(fabs(x), 1e10);  // beyond, ex2 = 0 (x = +-inf: erfc = 0 or 2)
  const double a = t + K, q = fma(2.0, t, 1.0);
  const double d = a * q;
  double r = rcp_approx(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double y = ((t - K) * q) * r;
  const double w = a * r;  // 1 / (1 + 2t)
  const double z = y * y;
  double ev = ERFC_POLY[22], od = ERFC_POLY[21];
#pragma unroll
  for (int j = 20; j >= 0; j -= 2) ev = fma(ev, z, ERFC_POLY[j]);
#pragma unroll
  for (int j = 19; j >= 1; j -= 2) od = fma(od, z, ERFC_POLY[j]);
  const double e = ex2 * (fma(od, y, ev) * w);
  return x < 0.0 ? 2.0 - e : e;
}

// first two half-space moments: sgn = +1 (u1 > 0) or -1 (u1 < 0)
template <class R>
TGKS_HD void half_seed(R U, R lam, double sgn, R& m0, R& m1) {
  const R isl = rsqrt_(lam);
  const R sl = lam * isl;
  const R ex = exp(-(lam * U) * U);
  m0 = 0.5 * erfc_exp(-sgn * (sl * U), ex);
  m1 = U * m0 + ((sgn * 0.28209479177387814347) * ex) * isl;  // 1/(2 sqrt(pi))
}

template <int D, class R>
struct MomSet {
  R m1[NM1];
  R mt[D > 1 ? D - 1 : 1][NMT];
  R xi1, xi2;  // <xi^2>, <xi^4>
};

template <int D, class R>
TGKS_HD R mono(const MomSet<D, R>& S, int i, int j, int k) {
  R v = S.m1[i];
  if (D >= 2) v = v * S.mt[0][j];
  if (D >= 3) v = v * S.mt[D >= 3 ? 1 : 0][k];
  return v;
}

// g[alpha] = <psi_alpha u1^i u2^j u3^k xi^(2l)>, l in {0, 1}
template <int D, class R>
TGKS_HD void gpsi(const MomSet<D, R>& S, int i, int j, int k, int l, R* g) {
  const R base = mono(S, i, j, k);
  g[0] = l == 0 ? base : base * S.xi1;
  g[1] = l == 0 ? mono(S, i + 1, j, k) : mono(S, i + 1, j, k) * S.xi1;
  if (D >= 2) g[2] = l == 0 ? mono(S, i, j + 1, k) : mono(S, i, j + 1, k) * S.xi1;
  if (D >= 3) g[D >= 3 ? 3 : 0] = l == 0 ? mono(S, i, j, k + 1) : mono(S, i, j, k + 1) * S.xi1;
  R e = mono(S, i + 2, j, k);
  if (D >= 2) e = e + mono(S, i, j + 2, k);
  if (D >= 3) e = e + mono(S, i, j, k + 2);
  g[D + 1] = l == 0 ? 0.5 * (e + base * S.xi1) : 0.5 * (e * S.xi1 + base * S.xi2);
}

// out[alpha] (+)= s * <psi_alpha a(psi) u1^i u2^j u3^k>
template <int D, bool ACC, class R>
TGKS_HD void mpsia(const MomSet<D, R>& S, const R* a, int i, int j, int k, R s, R* out) {
  constexpr int NC = D + 2;
  R g[NC], t[NC], r[NC];
  gpsi<D>(S, i, j, k, 0, g);
#pragma unroll
  for (int q = 0; q < NC; ++q) r[q] = a[0] * g[q];
  gpsi<D>(S, i + 1, j, k, 0, g);
#pragma unroll
  for (int q = 0; q < NC; ++q) r[q] += a[1] * g[q];
  if (D >= 2) {
    gpsi<D>(S, i, j + 1, k, 0, g);
#pragma unroll
    for (int q = 0; q < NC; ++q) r[q] += a[2] * g[q];
  }
  if (D >= 3) {
    gpsi<D>(S, i, j, k + 1, 0, g);
#pragma unroll
    for (int q = 0; q < NC; ++q) r[q] += a[D >= 3 ? 3 : 0] * g[q];
  }
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
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const R v = r[q] + ae * (t[q] + g[q]);
    if (ACC)
      out[q] += s * v;
    else
      out[q] = s * v;
  }
}

// closed-form solution a of <a psi> = b (per unit density) over the full
// Maxwellian (U, lambda), N = K + D.
template <int D, class R>
TGKS_HD void micro_solve(const Gas<D, R>& g, double N, const R* b, R* a) {
  R ub = R(0.0), u2 = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ub += g.U[d] * b[d + 1];
    u2 += g.U[d] * g.U[d];
  }
  const R lam = g.lam;
  const R aE = ((4.0 / N) * (lam * lam)) * ((2.0 * b[D + 1] - 2.0 * ub) + (u2 - N * g.h) * b[0]);
  R ua = R(0.0);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    a[d + 1] = (2.0 * lam) * (b[d + 1] - g.U[d] * b[0]) - g.U[d] * aE;
    ua += g.U[d] * a[d + 1];
  }
  a[D + 1] = aE;
  a[0] = (b[0] - ua) - (0.5 * aE) * (u2 + N * g.h);
}

template <int D, class R>
TGKS_HD void tangential_tables(const Gas<D, R>& g, MomSet<D, R>& S) {
#pragma unroll
  for (int d = 1; d < D; ++d) full_table(g.U[d], g.h, S.mt[d - 1], NMT);
}

template <int D, class R>
TGKS_HD void xi_moments(const Gas<D, R>& g, double K, MomSet<D, R>& S) {
  S.xi1 = K * g.h;
  S.xi2 = (K * (K + 2.0)) * (g.h * g.h);
}

// (i, j, k) exponents of u_d
TGKS_HD void unit(int d, int& i, int& j, int& k) {
  i = d == 0;
  j = d == 1;
  k = d == 2;
}

// heat-flux moment <phi X> from <u1 psi X> (f1) and <psi X> (f0):
// phi = (u1 - c1)(psi_E - c.u + |c|^2/2), c = U0 (face frame)
template <int D, class R>
TGKS_HD R heat_combine(const R* f1, const R* f0, const R* c) {
  R c2 = R(0.0), s1 = f1[D + 1], s0 = f0[D + 1];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c2 += c[d] * c[d];
    s1 -= c[d] * f1[d + 1];
    s0 -= c[d] * f0[d + 1];
  }
  s1 += (0.5 * c2) * f1[0];
  s0 += (0.5 * c2) * f0[0];
  return s1 - c[0] * s0;
}

// Directional derivatives of closed-form moments of a Maxwellian g(W).
// The derivative of g along a change dW of its conservative variables is
// g a(psi) with <a psi> = dW / rho, so every full-space moment of g a(psi)
// is the directional derivative of the corresponding moment of g:
//   rho <u_k psi a>      = J_k(W) dW     (Euler flux F_k = rho <u_k psi>)
//   rho <u_1 u_d psi a>  = dG_1d(W) dW   (G_1d = rho <u_1 u_d psi>)
// which replaces micro-slope solves and moment sums over the full space.
template <int D, class R>
struct Prim {
  R dU[D], dp, dh;
};

template <int D, class R>
TGKS_HD void prim_dir(const Gas<D, R>& g, double N, const R* dW, Prim<D, R>& o) {
  R udm = R(0.0), u2 = R(0.0);
#pragma unroll
  for (int e = 0; e < D; ++e) {
    o.dU[e] = (dW[e + 1] - g.U[e] * dW[0]) * g.irho;
    udm += g.U[e] * dW[e + 1];
    u2 += g.U[e] * g.U[e];
  }
  // p = (2/N)(E - rho |U|^2 / 2)
  o.dp = (2.0 / N) * ((dW[D + 1] - udm) + (0.5 * u2) * dW[0]);
  o.dh = (o.dp - g.h * dW[0]) * g.irho;
}

// out = J_k(W) dW, the Euler flux along frame axis k differentiated along dW
template <int D, class R>
TGKS_HD void euler_jvp(const Gas<D, R>& g, R E, int k, const R* dW, const Prim<D, R>& d, R* out) {
  const R p = g.rho * g.h;
  const R mk = g.rho * g.U[k];
  out[0] = dW[k + 1];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    R v = dW[k + 1] * g.U[e] + mk * d.dU[e];
    if (e == k) v += d.dp;
    out[e + 1] = v;
  }
  out[D + 1] = d.dU[k] * (E + p) + g.U[k] * (dW[D + 1] + d.dp);
}

// out = dG_1d(W) dW with G_1d = rho <u_1 u_d psi> (frame axis 0 normal):
//   alpha 0: rho U1 Ud + p [d=0]
//   alpha e: rho U1 Ud Ue + p (U1 [d=e] + Ud [e=0] + Ue [d=0])
//   alpha E: rho U1 Ud (|U|^2 + (N+4) h)/2 + [d=0] p (|U|^2 + (N+2) h)/2
template <int D, class R>
TGKS_HD void g1d_jvp(const Gas<D, R>& g, double N, int d, const R* dW, const Prim<D, R>& q, R* out) {
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
  const R rdA = dr * A + g.rho * dA;  // d(rho A)
  out[0] = d == 0 ? rdA + dp : rdA;
  const R rA = g.rho * A;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    R v = rdA * g.U[e] + rA * q.dU[e];
    if (d == e) v += dp * g.U[0] + p * q.dU[0];
    if (e == 0) v += dp * g.U[d] + p * q.dU[d];
    if (d == 0) v += dp * g.U[e] + p * q.dU[e];
    out[e + 1] = v;
  }
  const R Q = u2 + (N + 4.0) * g.h;
  const R dQ = 2.0 * udu + (N + 4.0) * q.dh;
  R vE = rdA * Q + rA * dQ;
  if (d == 0) {
    const R Rr = u2 + (N + 2.0) * g.h;
    const R dRr = 2.0 * udu + (N + 2.0) * q.dh;
    vE += dp * Rr + p * dRr;
  }
  out[D + 1] = 0.5 * vE;
}

// ---------------------------------------------------------------------------
// The Gauss-point flux in three pieces, for kernels that give the two sides
// of a Gauss point to two lanes: each lane evaluates its side's share of the
// equilibrium state (side_w0) and, once W0 is known, its side's shares of
// the slopes of W0 and of the non-equilibrium moments (side_part); the two
// shares are summed left + right and flux_combine adds the equilibrium part
// and the time integration.  gp_flux below evaluates the same arithmetic in
// one lane.
// ---------------------------------------------------------------------------
template <int D, class R>
struct SidePart {
  R dW0[D][D + 2];          // rho_s <psi a_d>_s: share of the slopes of W0 (Eq. 2.6)
  R S1[D + 2], S2[D + 2], S3[D + 2];  // rho_s <u1 psi>, sum_d <u1 u_d psi a_d>, <u1 psi A> over the half space
  R H1, H2, H3;             // their heat-flux moments (Navier-Stokes)
};

// gas state, half-space seeds and the side's share rho_s <psi>_s of W0;
// sgn = +1 for the left side (u1 > 0), -1 for the right side
template <int D, class R>
TGKS_HD void side_w0(const R* Ws, const FluxCfg& P, double sgn, Gas<D, R>& gs, R& h0, R& h1, R* w0) {
  constexpr int NC = D + 2;
  make_gas<D>(Ws, P.N, gs);
  half_seed(gs.U[0], gs.lam, sgn, h0, h1);
  MomSet<D, R> S;
  half_table(gs.U[0], gs.h, h0, h1, S.m1);
  tangential_tables<D>(gs, S);
  xi_moments<D>(gs, P.K, S);
  R g[NC];
  gpsi<D>(S, 0, 0, 0, 0, g);
#pragma unroll
  for (int q = 0; q < NC; ++q) w0[q] = gs.rho * g[q];
}

template <int D, bool NS, class R>
TGKS_HD void side_part(const Gas<D, R>& gs, R h0, R h1, const R* Ws, const R (*dW)[D + 2], const FluxCfg& P,
                       const Gas<D, R>& g0, SidePart<D, R>& o) {
  constexpr int NC = D + 2;
  const double N = P.N;
  MomSet<D, R> Sh;
  half_table(gs.U[0], gs.h, h0, h1, Sh.m1);
  tangential_tables<D>(gs, Sh);
  xi_moments<D>(gs, P.K, Sh);
  R a[D][NC];
  R Wt[NC];  // rho <(sum_d u_d a_d) psi> = sum_d J_d dW_d; A^s solves <A psi> = -that / rho
#pragma unroll
  for (int d = 0; d < D; ++d) {
    R b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) b[q] = dW[d][q] * gs.irho;
    micro_solve<D>(gs, N, b, a[d]);
    mpsia<D, false>(Sh, a[d], 0, 0, 0, gs.rho, o.dW0[d]);
    Prim<D, R> pd;
    prim_dir<D>(gs, N, dW[d], pd);
    R jv[NC];
    euler_jvp<D>(gs, Ws[D + 1], d, dW[d], pd, jv);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (d == 0)
        Wt[q] = jv[q];
      else
        Wt[q] += jv[q];
    }
  }
  R A[NC];
  {
    R b[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) b[q] = -(Wt[q] * gs.irho);
    micro_solve<D>(gs, N, b, A);
  }
  R g[NC];
  gpsi<D>(Sh, 1, 0, 0, 0, g);
  R v2[NC];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    int i, j, k;
    unit(d, i, j, k);
    if (d == 0)
      mpsia<D, false>(Sh, a[d], 1 + i, j, k, R(1.0), v2);
    else
      mpsia<D, true>(Sh, a[d], 1 + i, j, k, R(1.0), v2);
  }
  R v3[NC];
  mpsia<D, false>(Sh, A, 1, 0, 0, R(1.0), v3);
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    o.S1[q] = gs.rho * g[q];
    o.S2[q] = gs.rho * v2[q];
    o.S3[q] = gs.rho * v3[q];
  }
  o.H1 = o.H2 = o.H3 = R(0.0);
  if (NS) {
    R f0[NC], w2[NC], w3[NC];
    gpsi<D>(Sh, 0, 0, 0, 0, f0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      int i, j, k;
      unit(d, i, j, k);
      if (d == 0)
        mpsia<D, false>(Sh, a[d], i, j, k, R(1.0), w2);
      else
        mpsia<D, true>(Sh, a[d], i, j, k, R(1.0), w2);
    }
    mpsia<D, false>(Sh, A, 0, 0, 0, R(1.0), w3);
    o.H1 = gs.rho * heat_combine<D>(g, f0, g0.U);
    o.H2 = gs.rho * heat_combine<D>(v2, w2, g0.U);
    o.H3 = gs.rho * heat_combine<D>(v3, w3, g0.U);
  }
}

// Equilibrium part of Eq. 2.5 and the time integration over dt and dt/2,
// given W0, its gas state g0, the two sides' shares summed left + right
// (dW0, S1..S3, H1..H3) and the side pressures pl, pr (collision time).
template <int D, bool NS, class R>
TGKS_HD void flux_combine(const R* W0, const Gas<D, R>& g0, const SidePart<D, R>& T, R pl, R pr,
                          const FluxCfg& P, R dt, R* Fdt, R* Fh) {
  constexpr int NC = D + 2;
  const double N = P.N;
  const R(*dW0)[NC] = T.dW0;
  const R *S1 = T.S1, *S2 = T.S2, *S3 = T.S3;
  const R H1 = T.H1, H2 = T.H2, H3 = T.H3;
  // equilibrium part of Eq. 2.5, rho0-weighted moments in closed form:
  //   T1 = rho0 <u1 psi>_0 = F_1(W0)
  //   W0t = -sum_d J_d(W0) dW0_d = rho0 <Abar psi>_0 (compatibility, Eq. 2.7)
  //   T2 = rho0 sum_d <u1 u_d psi abar_d>_0 = sum_d dG_1d(W0) dW0_d
  //   T3 = rho0 <u1 psi Abar>_0 = J_1(W0) W0t
  R T1[NC], T2[NC], T3[NC], W0t[NC];
  {
    const R p0 = g0.rho * g0.h;
    const R E0 = W0[D + 1];
    T1[0] = W0[1];
#pragma unroll
    for (int e = 0; e < D; ++e) T1[e + 1] = W0[1] * g0.U[e] + (e == 0 ? p0 : R(0.0));
    T1[D + 1] = g0.U[0] * (E0 + p0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      Prim<D, R> pd;
      prim_dir<D>(g0, N, dW0[d], pd);
      R jv[NC], gv[NC];
      euler_jvp<D>(g0, E0, d, dW0[d], pd, jv);
      g1d_jvp<D>(g0, N, d, dW0[d], pd, gv);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (d == 0) {
          W0t[q] = -jv[q];
          T2[q] = gv[q];
        } else {
          W0t[q] -= jv[q];
          T2[q] += gv[q];
        }
      }
    }
    Prim<D, R> pt;
    prim_dir<D>(g0, N, W0t, pt);
    euler_jvp<D>(g0, E0, 0, W0t, pt, T3);
  }
  R G2 = R(0.0), G3 = R(0.0);  // heat-flux moments of the equilibrium part (the first vanishes)
  if (NS) {
    // <psi sum_d u_d abar_d>_0 = -<psi Abar>_0 by the compatibility condition
    R w2[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) w2[q] = -W0t[q];
    G2 = heat_combine<D>(T2, w2, g0.U);
    G3 = heat_combine<D>(T3, W0t, g0.U);
  }

  // collision time (Sec. 5 preamble); dt is the full step in both stages.
  // xh = -dt / (2 tau): e^{-dt/tau} = (e^{xh})^2, one expm1 serves both
  // intervals.
  const R S = pl + pr, A = fabs(pl - pr);
  R tau = R(0.0), xh = R(0.0);
  if (P.tau_mode == 1) {
    tau = P.mu * recip(g0.rho * g0.h) + (P.c2 * (A * recip(S))) * dt;
    xh = -(0.5 * dt) * recip(tau);
  } else if (P.tau_mode == 0) {
    // tau = (c1 + c2 A/S) dt = dt T/S with T = c1 S + c2 A; one reciprocal
    const R T = P.c1 * S + P.c2 * A;
    if (T > 0.0) {
      const R inv = recip(S * T);
      tau = dt * ((T * T) * inv);
      xh = -0.5 * ((S * S) * inv);
    }
  }
  R em = R(0.0);
  if (tau != 0.0) em = expm1(xh);

#pragma unroll
  for (int id = 0; id < 2; ++id) {
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
    const R C1 = dl - tau * ome;
    const R C2 = 2.0 * tt - (tau * dl) * (1.0 + e);
    const R C3 = (0.5 * dl) * dl - tau * dl + tt;
    const R C4 = tau * ome;
    const R C5 = (tau * dl) * e - 2.0 * tt;
    const R C6 = -tt;
    R* F = id == 0 ? Fdt : Fh;
#pragma unroll
    for (int q = 0; q < NC; ++q)
      F[q] = ((C1 * T1[q] + C2 * T2[q]) + C3 * T3[q]) + ((C4 * S1[q] + C5 * S2[q]) + C6 * S3[q]);
    if (NS) {
      const R q = (C2 * G2 + C3 * G3) + ((C4 * H1 + C5 * H2) + C6 * H3);
      F[NC - 1] += P.pr_fix * q;
    }
  }
}

// left + right sum of the two sides' shares, in that order
template <int D, class R>
TGKS_HD void side_sum(const SidePart<D, R>& l, const SidePart<D, R>& r, SidePart<D, R>& o) {
  constexpr int NC = D + 2;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
#pragma unroll
    for (int d = 0; d < D; ++d) o.dW0[d][q] = l.dW0[d][q] + r.dW0[d][q];
    o.S1[q] = l.S1[q] + r.S1[q];
    o.S2[q] = l.S2[q] + r.S2[q];
    o.S3[q] = l.S3[q] + r.S3[q];
  }
  o.H1 = l.H1 + r.H1;
  o.H2 = l.H2 + r.H2;
  o.H3 = l.H3 + r.H3;
}

// Time-integrated flux F(dt) and F(dt/2) at one Gauss point.
// Wl, Wr: states; dWl[d], dWr[d]: derivatives along frame axis d.
// Returns false when a state is non-physical.
template <int D, bool NS, class R>
TGKS_HD bool gp_flux(const R* Wl, const R* Wr, const R (*dWl)[D + 2], const R (*dWr)[D + 2], const FluxCfg& P,
                     R dt, R* Fdt, R* Fh) {
  constexpr int NC = D + 2;
  Gas<D, R> gl, gr, g0;
  R hl0, hl1, hr0, hr1, wl[NC], wr[NC], W0[NC];
  // equilibrium state by kinetic weighting (Eq. 2.6): rho_l <psi>_{>0} + rho_r <psi>_{<0}
  side_w0<D>(Wl, P, 1.0, gl, hl0, hl1, wl);
  side_w0<D>(Wr, P, -1.0, gr, hr0, hr1, wr);
#pragma unroll
  for (int q = 0; q < NC; ++q) W0[q] = wl[q] + wr[q];
  make_gas<D>(W0, P.N, g0);
  // side contributions: dW0 (Eq. 2.6), A^s (Eq. 2.7), and the moments of the
  // non-equilibrium part of Eq. 2.5 over the half space
  SidePart<D, R> L, Rt, T;
  side_part<D, NS>(gl, hl0, hl1, Wl, dWl, P, g0, L);
  side_part<D, NS>(gr, hr0, hr1, Wr, dWr, P, g0, Rt);
  side_sum<D>(L, Rt, T);
  flux_combine<D, NS>(W0, g0, T, gl.rho * gl.h, gr.rho * gr.h, P, dt, Fdt, Fh);
  return gl.ok && gr.ok && g0.ok;
}

// The Gauss-point flux with a separately reconstructed equilibrium (WENO-Z
// and TENO5 GKS, Sec. 3.1): the slopes of W0 along every frame axis are
// given (dW0), and so is W0 itself when W0in is not null (2-D: the
// tangential reconstruction of the face segments' equilibrium states);
// otherwise W0 is the kinetic weighting of the two sides (Eq. 2.6).
template <int D, bool NS, class R>
TGKS_HD bool gp_flux_eq(const R* Wl, const R* Wr, const R (*dWl)[D + 2], const R (*dWr)[D + 2], const R* W0in,
                        const R (*dW0)[D + 2], const FluxCfg& P, R dt, R* Fdt, R* Fh) {
  constexpr int NC = D + 2;
  Gas<D, R> gl, gr, g0;
  R hl0, hl1, hr0, hr1, wl[NC], wr[NC], W0[NC];
  side_w0<D>(Wl, P, 1.0, gl, hl0, hl1, wl);
  side_w0<D>(Wr, P, -1.0, gr, hr0, hr1, wr);
#pragma unroll
  for (int q = 0; q < NC; ++q) W0[q] = W0in ? W0in[q] : wl[q] + wr[q];
  make_gas<D>(W0, P.N, g0);
  SidePart<D, R> L, Rt, T;
  side_part<D, NS>(gl, hl0, hl1, Wl, dWl, P, g0, L);
  side_part<D, NS>(gr, hr0, hr1, Wr, dWr, P, g0, Rt);
  side_sum<D>(L, Rt, T);
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int q = 0; q < NC; ++q) T.dW0[d][q] = dW0[d][q];
  flux_combine<D, NS>(W0, g0, T, gl.rho * gl.h, gr.rho * gr.h, P, dt, Fdt, Fh);
  return gl.ok && gr.ok && g0.ok;
}

// ---------------------------------------------------------------------------
// Boundary index map (ghost cells): periodic, transmissive (copy of the
// nearest cell), reflective (mirror image; flip = 1: the momentum normal to
// the wall changes sign) or a no-slip adiabatic wall (mirror image; flip =
// 2: every momentum component changes sign).
// ---------------------------------------------------------------------------
constexpr int BC_NOSLIP = 3;  // boundary kind of the no-slip adiabatic wall
constexpr int BC_PRESCRIBED = 4;  // boundary kind of given states (resolved before the map)

TGKS_HD int map_index(int i, int n, int bclo, int bchi, int& flip) {
  if (i >= 0 && i < n) return i;
  const int bc = i < 0 ? bclo : bchi;
  if (bc == 0) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  if (bc == 1) return i < 0 ? 0 : n - 1;
  flip ^= bc == BC_NOSLIP ? 2 : 1;
  // mirror image; cells farther than n outside are never used by a face and
  // are clamped into the domain so that every load stays in bounds
  const int r = i < 0 ? -1 - i : 2 * n - 1 - i;
  return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

}  // namespace tgks
