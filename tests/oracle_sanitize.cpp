// Runs every entry point of the oracle on small 1-D, 2-D and 3-D grids with
// all boundary kinds, under AddressSanitizer and UndefinedBehaviorSanitizer
// (built and run by test_oracle_sanitize.py).  Any out-of-bounds access,
// use of uninitialised memory through UB, or signed overflow aborts.
#include "../oracle/gks_oracle.cpp"

#include <cstdio>
#include <vector>

static orc_params params(int D, int n, int bc, int tau, double mu) {
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.ndim = D;
  for (int d = 0; d < 3; ++d) {
    p.n[d] = d < D ? n + d : 1;
    p.dx[d] = d < D ? 1.0 / (n + d) : 1.0;
    p.bc_lo[d] = p.bc_hi[d] = bc;
  }
  p.gamma = 1.4;
  p.mu = mu;
  p.prandtl = mu > 0 ? 0.72 : 1.0;
  p.tau_mode = tau;
  p.c1 = 0.01;
  p.c2 = 1.0;
  p.ct1 = p.ct1_tan = 1e-7;
  p.ct2 = p.ct2_tan = 1e-5;
  p.eps = 1e-40;
  p.q = 7;
  // prescribed sides: states A, B and a moving line on every side, each far
  // kind once
  const double A[5] = {2.0, 0.4, -0.2, 0.1, 6.0}, B[5] = {1.0, 0.0, 0.1, 0.0, 2.5};
  for (int c = 0; c < D + 1; ++c) {
    p.bc_state[0][c] = A[c];
    p.bc_state[1][c] = B[c];
  }
  p.bc_state[0][D + 1] = A[4];
  p.bc_state[1][D + 1] = B[4];
  const int far[4] = {2, 1, 4, 2};
  for (int d = 0; d < 2; ++d)
    for (int e = 0; e < 2; ++e) {
      p.bc_line[d][e][0] = 0.3 + 0.1 * e;
      p.bc_line[d][e][1] = 0.5;
      p.bc_line[d][e][2] = 1.0;
      p.bc_far[d][e] = far[2 * d + e];
    }
  return p;
}

static std::vector<double> field(const orc_params& p, int jump) {
  const int D = p.ndim, nc = D + 2;
  const long n = (long)p.n[0] * p.n[1] * p.n[2];
  std::vector<double> W(nc * n);
  for (long c = 0; c < n; ++c) {
    const int i = (int)(c % p.n[0]), j = (int)((c / p.n[0]) % p.n[1]), k = (int)(c / ((long)p.n[0] * p.n[1]));
    const double x = (i + 0.5) / p.n[0], y = (j + 0.5) / p.n[1], z = (k + 0.5) / p.n[2];
    double rho = 1.0 + 0.2 * std::sin(6.283 * x + 1.0) * std::cos(6.283 * y) + 0.1 * std::sin(6.283 * z);
    double pr = 1.0 + 0.2 * std::cos(6.283 * (x + y + z));
    if (jump && x > 0.5) {
      rho *= 2.0;
      pr *= 1.5;
    }
    const double u[3] = {0.3 * std::sin(6.283 * y), -0.2 * std::cos(6.283 * x), 0.1};
    double ke = 0.0;
    W[c] = rho;
    for (int d = 0; d < D; ++d) {
      W[(d + 1) * n + c] = rho * u[d];
      ke += u[d] * u[d];
    }
    W[(D + 1) * n + c] = pr / 0.4 + 0.5 * rho * ke;
  }
  return W;
}

int main() {
  int cases = 0;
  for (int D = 1; D <= 3; ++D)
    for (int bc = 0; bc <= 4; ++bc)
      for (int tau = 0; tau <= 1; ++tau) {
        if (bc == 4 && D == 3) continue;  // prescribed sides: 1-D and 2-D grids
        const int n = D == 3 ? 3 : (D == 2 ? 7 : 13);
        orc_params p = params(D, n, bc, tau, tau == 1 ? 1e-3 : 0.0);
        std::vector<double> W = field(p, bc != 0), Wo(W.size()), Wo2(W.size()), Ws(W.size()), dW(W.size()),
            dWo(W.size());
        for (size_t i = 0; i < W.size(); ++i) dW[i] = 1e-3 * std::sin(0.37 * i);
        std::vector<uint8_t> flags(orc_flag_bytes(&p));
        double dt = 0.0;
        if (orc_cfl_dt(&p, W.data(), 0.5, &dt) != 0) return 2;
        long nfb = 0;
        p.fallback = D <= 2 && tau == 1 ? 1 : 0;
        if (orc_step(&p, W.data(), Wo.data(), dt, flags.data(), Ws.data(), 0.1, &nfb) < 0) return 3;
        p.fallback = 0;
        if (orc_step_dual(&p, W.data(), dW.data(), Wo2.data(), dWo.data(), dt) < 0) return 4;
        std::vector<double> Wr(W);
        double t = 0.0;
        int steps = 0;
        if (orc_run(&p, Wr.data(), 2, 0.5, 0.0, 0.0, &t, &steps, 0.05) < 0) return 5;
        // one Gauss-point flux and its derivative in the face frame
        double Wl[5] = {1.0, 0.1, 0.05, 0.02, 2.6}, Wrr[5] = {0.9, -0.1, 0.0, 0.01, 2.4};
        double dWl[15], dWr[15], tW[5], tdW[15], F[10], dF[10], W0[5], dW0[15];
        for (int i = 0; i < 15; ++i) {
          dWl[i] = 0.01 * (i + 1);
          dWr[i] = -0.01 * i;
          tdW[i] = 0.1;
        }
        for (int i = 0; i < 5; ++i) tW[i] = 0.2;
        const double deltas[2] = {dt, 0.5 * dt};
        if (orc_gp_flux(&p, Wl, Wrr, dWl, dWr, dt, 2, deltas, F, W0, dW0) < 0) return 6;
        if (orc_gp_flux_dual(&p, Wl, Wrr, dWl, dWr, tW, tW, tdW, tdW, dt, 2, deltas, F, dF) < 0) return 7;
        ++cases;
      }
  // reconstruction and moment entry points
  double Q[5] = {1.0, 1.1, 1.3, 0.9, 1.0}, out[8], beta[4];
  orc_beta(Q, beta);
  (void)orc_teno_select(Q, 1e-7, 1e-5, 1e-40, 7);
  orc_teno_face(Q, 1e-7, 1e-5, 1e-40, 7, out);
  orc_teno_gauss(Q, 1e-7, 1e-5, 1e-40, 7, out);
  for (int flag = 0; flag < 16; ++flag) orc_teno_eval(Q, flag, flag & 1, out);
  double mom[32];
  for (int kind = 0; kind < 3; ++kind) orc_moments(0.3, 1.7, kind, mom);
  std::printf("oracle sanitizer run: %d grid cases\n", cases);
  return 0;
}
