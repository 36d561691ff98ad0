// tgks_adjoint_kernels.hpp -- reverse of one S2O4 step (1-D and 2-D) with the
// time step and the stencil selections frozen (the reconstruction is then a
// linear map; Sec. 4.2 selections are recomputed from the same state bits as
// in the forward step and therefore identical).
//
// One flux stage in direction AX is reversed by three gathers:
//   face kernel   per face: cotangents of the two Gauss-point fluxes from the
//                 cell cotangents on both sides of the face, the forward
//                 reconstruction recomputed, and the reverse of the flux
//                 (tgks_adjoint.hpp); out: cotangents of the tangential
//                 reconstruction's point values (2-D) or of the normal
//                 reconstruction's face values (1-D), and the tangential flags
//   tangential    per normal-reconstructed cell: the transposed tangential
//                 reconstruction gathered from the five faces that used it
//   normal        per interior cell: the transposed normal reconstruction of
//                 the five cells that used it, gathered over every ghost
//                 image of the cell (periodic, transmissive and reflective
//                 index maps, momentum sign of a mirror image)
// The face cotangents follow from the flux-difference update: with
// W_i -= (F_{i+1/2} - F_{i-1/2}) / dx, the cotangent of F_{i+1/2} is
// (X_{i+1} - X_i) / dx for a cell cotangent X (zero outside the domain).
#pragma once
#include "tgks_adjoint.hpp"
#include "tgks_kernels.hpp"

namespace tgks {

struct AdjArgs {
  Geom g;
  FluxCfg fc;
  TenoCfg tn, tt;
  const double* W;   // state the stage's fluxes were computed from
  const double* X;   // cell cotangents (coefficients cx) and
  const double* Y;   // (coefficients cy), Y may be null
  double cx_dt, cx_h, cy_dt, cy_h;  // F(dt), F(dt/2) face cotangent = c_X D^T X + c_Y D^T Y
  const double* dt;
  double* GB;        // 2-D: Gauss-point cotangents [side][c][6][faces]
  uint8_t* TF;       // 2-D: tangential flags [side][W, W_n][c][faces]
  double* NRB;       // normal-reconstruction cotangents [c][4][ext cells]
  uint8_t* NF;       // normal selections of the extended cells [c][ext cells]
  const double* base0;
  const double* base1;
  double* out;
};

// extended normal-reconstruction cells: AX index in [-1, n_AX], tangential
// index in [-2, n_T + 2) (2-D), stored [c][slot][cells] with the x index
// fastest: [t + 2][i + 1] for x faces, [i + 1][t + 2] for y faces
__device__ __forceinline__ long long ext_count(const Geom& g, int ax) {
  const int ne = g.n[ax] + 2;
  return g.D == 1 ? (long long)ne : (long long)ne * (g.n[1 - ax] + 4);
}

__device__ __forceinline__ long long ext_index(const Geom& g, int ax, int i, int t) {
  if (g.D == 1) return (long long)(i + 1);
  return ax == 0 ? (long long)(t + 2) * (g.n[0] + 2) + (i + 1) : (long long)(i + 1) * (g.n[0] + 4) + (t + 2);
}

// cotangent of component c of the flux on the face between cells lo and hi
// (linear cell indices, -1 when outside the domain) along axis ax
__device__ __forceinline__ void face_cot(const AdjArgs& a, int c, long long lo, long long hi, double idx, double& fdt,
                                         double& fh) {
  const long long o = (long long)c * a.g.ncell;
  const double xhi = hi >= 0 ? a.X[o + hi] : 0.0, xlo = lo >= 0 ? a.X[o + lo] : 0.0;
  const double dX = (xhi - xlo) * idx;
  fdt = a.cx_dt * dX;
  fh = a.cx_h * dX;
  if (a.Y) {
    const double yhi = hi >= 0 ? a.Y[o + hi] : 0.0, ylo = lo >= 0 ? a.Y[o + lo] : 0.0;
    const double dY = (yhi - ylo) * idx;
    fdt += a.cy_dt * dY;
    fh += a.cy_h * dY;
  }
}

// ---------------------------------------------------------------------------
// 1-D face kernel: one thread per face; writes the cotangents of the normal
// reconstruction's face values of the cells on both sides.
// ---------------------------------------------------------------------------
template <bool NS>
__global__ __launch_bounds__(128) void adj_face1d_kernel(AdjArgs a) {
  const double dt = *a.dt;
  const int n = a.g.n[0];
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f > n) return;
  const double idx = 1.0 / a.g.dx[0];
  double Wl[3], Wr[3], dWl[1][3], dWr[1][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double Q[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) Q[r] = load_cell(a.g, a.W, c, f - 3 + r, 0, 0);
    double o[4];
    teno_face(Q, teno_flag<SEL_FILTER>(Q, a.tn), o);
    Wl[c] = o[2];
    dWl[0][c] = o[3] * idx;
    teno_face(Q + 1, teno_flag<SEL_FILTER>(Q + 1, a.tn), o);
    Wr[c] = o[0];
    dWr[0][c] = o[1] * idx;
  }
  double Fdtb[3], Fhb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    face_cot(a, c, f >= 1 ? f - 1 : -1, f < n ? f : -1, idx, Fdtb[c], Fhb[c]);
  wall_fluxes<3>(a.g, 0, f, Fdtb, Fhb);  // transpose of the zero wall fluxes
  double Wlb[3], Wrb[3], dWlb[1][3], dWrb[1][3];
  if (dt > 0.0) {
    gp_flux_vjp<1, NS, double>(Wl, Wr, dWl, dWr, a.fc, dt, Fdtb, Fhb, Wlb, Wrb, dWlb, dWrb);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) Wlb[c] = Wrb[c] = dWlb[0][c] = dWrb[0][c] = 0.0;
  }
  const long long ne = ext_count(a.g, 0);
  const long long il = ext_index(a.g, 0, f - 1, 0), ir = ext_index(a.g, 0, f, 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double* B = a.NRB + (long long)c * 4 * ne;
    B[2 * ne + il] = Wlb[c];
    B[3 * ne + il] = dWlb[0][c] * idx;
    B[0 * ne + ir] = Wrb[c];
    B[1 * ne + ir] = dWrb[0][c] * idx;
    // the outer face values of the two outermost extended cells feed no face
    if (f == 0) B[0 * ne + il] = B[1 * ne + il] = 0.0;
    if (f == n) B[2 * ne + ir] = B[3 * ne + ir] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 2-D face kernel: a block owns TN x TT faces, stages the cells and their
// normal reconstruction in LDS as the forward kernel does; lanes 2k and 2k+1
// share face k: lane m reconstructs side m along the face at both Gauss
// points (and writes that side's tangential selections), hands the partner
// its side at the partner's Gauss point, and reverses the flux at Gauss
// point m.
// ---------------------------------------------------------------------------
constexpr int ATN = 8, ATT = 16;

template <int AX, bool NS>
__global__ __launch_bounds__(2 * ATN * ATT) void adj_face2d_kernel(AdjArgs a) {
  constexpr int TN = ATN, TT = ATT, NT = 2 * TN * TT;
  constexpr int NC = 4;
  constexpr int LN = TN + 5, LT = TT + 4, RN = TN + 1;
  __shared__ double sW[NC][LT][LN];
  __shared__ double sR[NC][LT][RN][4];
  const double dt = *a.dt;
  const Geom& g = a.g;
  const int TA = 1 - AX;
  const int nN = g.n[AX], nT = g.n[TA];
  const int f0 = blockIdx.x * TN, t0 = blockIdx.y * TT;
  const int tid = threadIdx.x;
  // one thread per staged cell: one index map, four component loads
  for (int L = tid; L < LN * LT; L += NT) {
    int nl, tl;
    if (AX == 0) {
      nl = L % LN;
      tl = L / LN;
    } else {
      tl = L % LT;
      nl = L / LT;
    }
    const int pn = f0 - 3 + nl, pt = t0 - 2 + tl;
    int m0, m1, m2;
    const long long off = cell_offset(g, AX == 0 ? pn : pt, AX == 0 ? pt : pn, 0, m0, m1, m2);
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = a.W[(long long)c * g.ncell + off];
#pragma unroll
    for (int c = 0; c < NC; ++c) sW[c][tl][nl] = cell_flip(g, c, m0, m1, m2) ? -v[c] : v[c];
  }
  __syncthreads();
  const double idn = 1.0 / g.dx[AX];
  for (int L = tid; L < NC * LT * RN; L += NT) {
    const int nr = L % RN;
    const int tl = (L / RN) % LT;
    const int c = L / (RN * LT);
    const double* Q = &sW[c][tl][nr];
    double o[4];
    teno_face(Q, teno_flag<SEL_FILTER>(Q, a.tn), o);
    sR[c][tl][nr][0] = o[0];
    sR[c][tl][nr][1] = o[1] * idn;
    sR[c][tl][nr][2] = o[2];
    sR[c][tl][nr][3] = o[3] * idn;
  }
  __syncthreads();
  const int m = tid & 1;
  const int fi = tid >> 1;
  const int fn = fi % TN, ft = fi / TN;
  const int f = f0 + fn, t = t0 + ft;
  if (f > nN || t >= nT) return;  // both lanes of a face leave together
  const int perm[NC] = {0, 1 + AX, 1 + TA, 3};
  const long long nf = face_count(g, AX);
  const long long fidx = AX == 0 ? (long long)t * (g.n[0] + 1) + f : (long long)f * g.n[0] + t;
  const double idt = 1.0 / g.dx[TA];
  // own side m along the face; the partner's side at this Gauss point
  double Wg[2][NC], Dg[2][2][NC];  // [side][q], [side][axis n/t][q]
  {
    const int nr = m == 0 ? fn : fn + 1;
    const int vo = m == 0 ? 2 : 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = perm[q];
      double Qw[5], Qn[5], v[2], dv[2], vn[2], dn[2];
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        Qw[r] = sR[c][ft + r][nr][vo];
        Qn[r] = sR[c][ft + r][nr][vo + 1];
      }
      const unsigned fw = teno_flag<SEL_FILTER>(Qw, a.tt), fq = teno_flag<SEL_FILTER>(Qn, a.tt);
      a.TF[((long long)(m * 2 + 0) * NC + c) * nf + fidx] = (uint8_t)fw;
      a.TF[((long long)(m * 2 + 1) * NC + c) * nf + fidx] = (uint8_t)fq;
      teno_gauss(Qw, fw, v, dv);
      teno_gauss(Qn, fq, vn, dn);
      const double sv = m ? v[0] : v[1], sd = m ? dv[0] : dv[1], sn = m ? vn[0] : vn[1];
      const double rv = lane_xor<1>(sv), rd = lane_xor<1>(sd), rn = lane_xor<1>(sn);
      const double ov = m ? v[1] : v[0], od = m ? dv[1] : dv[0], on = m ? vn[1] : vn[0];
      Wg[0][q] = m == 0 ? ov : rv;
      Wg[1][q] = m == 0 ? rv : ov;
      Dg[0][1][q] = (m == 0 ? od : rd) * idt;
      Dg[1][1][q] = (m == 0 ? rd : od) * idt;
      Dg[0][0][q] = m == 0 ? on : rn;
      Dg[1][0][q] = m == 0 ? rn : on;
    }
  }
  // face cotangents (global components), Gauss weight 1/2
  double Fdtb[NC], Fhb[NC];
  {
    const long long cell_hi = AX == 0 ? (long long)t * g.n[0] + f : (long long)f * g.n[0] + t;
    const long long stride = AX == 0 ? 1 : g.n[0];
    const long long lo = f >= 1 ? cell_hi - stride : -1, hi = f < nN ? cell_hi : -1;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      double x, y;
      face_cot(a, perm[q], lo, hi, idn, x, y);
      Fdtb[q] = 0.5 * x;
      Fhb[q] = 0.5 * y;
    }
    wall_fluxes<NC>(g, AX, f, Fdtb, Fhb);  // transpose of the zero wall fluxes
  }
  double Wb[2][NC], Db[2][2][NC];
  if (dt > 0.0) {
    gp_flux_vjp<2, NS, double>(Wg[0], Wg[1], Dg[0], Dg[1], a.fc, dt, Fdtb, Fhb, Wb[0], Wb[1], Db[0], Db[1]);
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < NC; ++q) Wb[s][q] = Db[s][0][q] = Db[s][1][q] = 0.0;
  }
  double* GB = a.GB;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const long long base = ((long long)(s * NC + perm[q]) * 6) * nf + fidx;
      GB[base + (long long)(0 + m) * nf] = Wb[s][q];
      GB[base + (long long)(2 + m) * nf] = Db[s][1][q] * idt;
      GB[base + (long long)(4 + m) * nf] = Db[s][0][q];
    }
}

// ---------------------------------------------------------------------------
// 2-D tangential transpose: one thread per extended cell and component.
// ---------------------------------------------------------------------------
template <int AX>
__global__ __launch_bounds__(256) void adj_tan2d_kernel(AdjArgs a) {
  constexpr int NC = 4;
  const Geom& g = a.g;
  const int TA = 1 - AX;
  const int nN = g.n[AX], nT = g.n[TA];
  const long long ne = ext_count(g, AX);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * NC) return;
  const int c = (int)(id / ne);
  const long long e = id % ne;  // == ext_index(g, AX, i, r)
  const int i = AX == 0 ? (int)(e % (nN + 2)) - 1 : (int)(e / (nT + 4)) - 1;
  const int r = AX == 0 ? (int)(e / (nN + 2)) - 2 : (int)(e % (nT + 4)) - 2;
  const long long nf = face_count(g, AX);
  const double idn = 1.0 / g.dx[AX];
  double o[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    // side 1 of face i uses the cell's low-face values; side 0 of face i + 1
    // its high-face values
    const int fn = s == 1 ? i : i + 1;
    if (fn < 0 || fn > nN) continue;
    double accv = 0.0, accn = 0.0;
    for (int k = 0; k < 5; ++k) {
      const int ft = r + 2 - k;  // face whose stencil slot k is this cell
      if (ft < 0 || ft >= nT) continue;
      const long long fidx = AX == 0 ? (long long)ft * (g.n[0] + 1) + fn : (long long)fn * g.n[0] + ft;
      const unsigned fw = a.TF[((long long)(s * 2 + 0) * NC + c) * nf + fidx];
      const unsigned fq = a.TF[((long long)(s * 2 + 1) * NC + c) * nf + fidx];
      double Q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      Q[k] = 1.0;
      double v[2], d[2], vn[2], dn[2];
      teno_gauss(Q, fw, v, d);
      teno_gauss(Q, fq, vn, dn);
      const long long base = ((long long)(s * NC + c) * 6) * nf + fidx;
      accv += (v[0] * a.GB[base] + v[1] * a.GB[base + nf]) + (d[0] * a.GB[base + 2 * nf] + d[1] * a.GB[base + 3 * nf]);
      accn += vn[0] * a.GB[base + 4 * nf] + vn[1] * a.GB[base + 5 * nf];
    }
    const int vo = s == 1 ? 0 : 2;
    o[vo] = accv;
    o[vo + 1] = accn * idn;
  }
  double* B = a.NRB + (long long)c * 4 * ne + e;
#pragma unroll
  for (int k = 0; k < 4; ++k) B[k * ne] = o[k];
}

// Normal selections of every extended cell (AX index in [-1, n_AX], the
// tangential index in [-2, n_T + 2) in 2-D), one thread per cell and
// component: the same selection as the forward reconstruction.
template <int D, int AX>
__global__ __launch_bounds__(256) void adj_nflags_kernel(AdjArgs a) {
  constexpr int NC = D + 2;
  const Geom& g = a.g;
  const long long ne = ext_count(g, AX);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * NC) return;
  const int c = (int)(id / ne);
  const long long e = id % ne;
  const int nN = g.n[AX];
  int i, r = 0;
  if (D == 1) {
    i = (int)e - 1;
  } else {
    const int nT = g.n[1 - AX];
    i = AX == 0 ? (int)(e % (nN + 2)) - 1 : (int)(e / (nT + 4)) - 1;
    r = AX == 0 ? (int)(e / (nN + 2)) - 2 : (int)(e % (nT + 4)) - 2;
  }
  double Q[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int pa = i - 2 + q;
    Q[q] = D == 1 ? load_cell(g, a.W, c, pa, 0, 0) : load_cell(g, a.W, c, AX == 0 ? pa : r, AX == 0 ? r : pa, 0);
  }
  a.NF[(long long)c * ne + e] = (uint8_t)teno_flag<SEL_FILTER>(Q, a.tn);
}

// preimages of interior index x under the boundary index map among the
// candidates x and the ghost indices -G..-1, n..n+G-1; returns the count
template <int G>
__device__ __forceinline__ int preimages(int x, int n, int bclo, int bchi, int* idx, int* flip) {
  int cnt = 0;
  for (int k = 0; k <= 2 * G; ++k) {
    const int cand = k == 0 ? x : (k <= G ? -k : n + (k - G - 1));
    int fl = 0;
    if (map_index(cand, n, bclo, bchi, fl) == x) {
      idx[cnt] = cand;
      flip[cnt] = fl;
      ++cnt;
    }
  }
  return cnt;
}

// ---------------------------------------------------------------------------
// Normal transpose and ghost map, 1-D and 2-D: one thread per interior cell
// and component; out = base0 + base1 + gathered cotangent.
// ---------------------------------------------------------------------------
template <int D, int AX>
__global__ __launch_bounds__(256) void adj_normal_kernel(AdjArgs a) {
  constexpr int NC = D + 2;
  const Geom& g = a.g;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.ncell * NC) return;
  const int c = (int)(id / g.ncell);
  const long long cell = id % g.ncell;
  const int x = (int)(cell % g.n[0]);
  const int y = D >= 2 ? (int)(cell / g.n[0]) : 0;
  const int TA = 1 - AX;
  const int xn = AX == 0 ? x : y;  // index along AX
  const int xt = AX == 0 ? y : x;  // index along the tangential axis
  const int nN = g.n[AX];
  const long long ne = ext_count(g, AX);
  int pn[7], fn_[7], pt[5], ft_[5];
  const int cn = preimages<3>(xn, nN, g.bclo[AX], g.bchi[AX], pn, fn_);
  int ct = 1;
  pt[0] = 0;
  ft_[0] = 0;
  if (D == 2) ct = preimages<2>(xt, g.n[TA], g.bclo[TA], g.bchi[TA], pt, ft_);
  double acc = 0.0;
  for (int u = 0; u < ct; ++u) {
    const int r = pt[u];
    for (int w = 0; w < cn; ++w) {
      const int ip = pn[w];
      // sign of the image: the momentum normal to a reflective wall, every
      // momentum component behind a no-slip wall
      const bool mom = c >= 1 && c <= D;
      bool neg = (c == 1 + AX && fn_[w] == 1) ^ (mom && fn_[w] == 2);
      if (D == 2) neg ^= (c == 1 + TA && ft_[u] == 1) ^ (mom && ft_[u] == 2);
      double s = 0.0;
      for (int k = 0; k < 5; ++k) {
        const int i = ip + 2 - k;  // cell whose normal stencil slot k is ip
        if (i < -1 || i > nN) continue;
        const long long ei = ext_index(g, AX, i, r);
        const unsigned fl = a.NF[(long long)c * ne + ei];
        double E[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, o[4];
        E[k] = 1.0;
        teno_face(E, fl, o);
        const double* B = a.NRB + (long long)c * 4 * ne + ei;
        s += (o[0] * B[0] + o[1] * B[ne]) + (o[2] * B[2 * ne] + o[3] * B[3 * ne]);
      }
      acc += neg ? -s : s;
    }
  }
  double v = acc;
  if (a.base0) v += a.base0[id];
  if (a.base1) v += a.base1[id];
  a.out[id] = v;
}

}  // namespace tgks
