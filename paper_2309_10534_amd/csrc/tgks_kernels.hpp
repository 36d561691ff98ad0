// tgks_kernels.hpp -- HIP kernels of one S2O4 step of the TENO-D GKS (gfx950).
//
// Per stage and direction a face kernel produces, for every face, the
// Gauss-point averaged time-integrated fluxes combined as the S2O4 update
// needs them (Sec. 2.2):
//   stage 1:  FA = F(W^n, dt/2),  FB = 8/3 F(W^n, dt/2) - 1/3 F(W^n, dt)
//   stage 2:  FA = 4/3 F(W*, dt) - 8/3 F(W*, dt/2)
// so that  W* = W^n - sum_d D_d FA / dx_d,  P = W^n - sum_d D_d FB / dx_d,
// W^{n+1} = P - sum_d D_d FA* / dx_d, algebraically the update of Sec. 2.2.
// The update kernels apply the flux differences; the stage-2 update also
// reduces the CFL time step of the new state (Sec. 5 preamble).
#pragma once
#include "tgks_device.hpp"

namespace tgks {

struct Geom {
  int D;
  int n[3];
  double dx[3];
  int bclo[3], bchi[3];
  long long ncell;
};

// Prescribed sides of 1-D and 2-D grids: a ghost cell centred at s along
// the other axis (0 in 1-D) and r along the side's axis holds A where
// s < (s0 + s_n r) + s_t t, beyond the line B (far == BC_PRESCRIBED) or the
// transmissive / reflective image (far == 1 / 2).
struct Prescribed {
  int on;               // some side is prescribed
  int far[2][2];        // [axis][end]
  double A[4], B[4];    // global component order
  double line[2][2][3]; // [axis][end]: s0, s_n, s_t
};

// value of lane (lane ^ MASK), MASK = 1 or 2, by a DPP quad permute (a
// VALU move; no LDS instruction, unlike a general lane shuffle)
template <int MASK>
__device__ __forceinline__ int lane_xor(int v) {
  static_assert(MASK == 1 || MASK == 2, "quad permutes only");
  return __builtin_amdgcn_mov_dpp(v, MASK == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int MASK>
__device__ __forceinline__ double lane_xor(double v) {
  const int lo = lane_xor<MASK>(__double2loint(v)), hi = lane_xor<MASK>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// value of lane 7 - i within the lane's group of eight (DPP half-row
// mirror): for a value that is the same in the four lanes of each quad, the
// other quad's value, as lane ^ 4 would give
__device__ __forceinline__ double other_quad(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x141, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x141, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

struct StageArgs {
  Geom g;
  FluxCfg fc;
  TenoCfg tn;  // normal reconstruction
  TenoCfg tt;  // tangential reconstruction
  SchemeCfg sc;  // constants of the comparison schemes (WENO-AO, TENO5, WENO-Z)
  const double* W;
  double* FA;
  double* FB;
  const double* dt;
  unsigned long long* fail;
  uint8_t* nflags;  // normal flags [D][nc][cells] or null
  uint8_t* tflags;  // tangential flags of this direction or null
  const double* R;  // 3-D: normal reconstruction of this direction
  double* Rout;
  double gamma;     // ratio of specific heats (characteristic variables)
  Prescribed pb;    // prescribed sides
  double t0;        // time of W (prescribed states) is t0 + *tclk (tclk may be null)
  const double* tclk;
  int fallback;     // 1: first-order fallback at non-physical Gauss-point states
  unsigned long long* fbc;  // fallback counter, or null (not counted)
};

__device__ __forceinline__ long long face_count(const Geom& g, int ax) {
  long long c = 1;
  for (int d = 0; d < 3; ++d) c *= (long long)(d == ax ? g.n[d] + 1 : g.n[d]);
  return c;
}

// offset of the cell (i, j, k) within a component plane, ghost cells by the
// boundary index map; f0..f2 receive the mirror kinds along each axis
__device__ __forceinline__ long long cell_offset(const Geom& g, int i, int j, int k, int& f0, int& f1, int& f2) {
  f0 = f1 = f2 = 0;
  const int ii = map_index(i, g.n[0], g.bclo[0], g.bchi[0], f0);
  const int jj = g.D >= 2 ? map_index(j, g.n[1], g.bclo[1], g.bchi[1], f1) : 0;
  const int kk = g.D >= 3 ? map_index(k, g.n[2], g.bclo[2], g.bchi[2], f2) : 0;
  return ((long long)kk * g.n[1] + jj) * g.n[0] + ii;
}

// whether component c (global order) changes sign at a mirrored cell: a
// reflective wall negates the momentum normal to it, a no-slip wall every
// momentum component
__device__ __forceinline__ bool cell_flip(const Geom& g, int c, int f0, int f1, int f2) {
  if (c < 1 || c > g.D) return false;
  const int fo = c == 1 ? f0 : (c == 2 ? f1 : f2);
  return (fo == 1) ^ (f0 == 2) ^ (f1 == 2) ^ (f2 == 2);
}

// value of component c (global order) of the cell (i, j, k), ghost cells by
// the boundary index map
__device__ __forceinline__ double load_cell(const Geom& g, const double* W, int c, int i, int j, int k) {
  int f0, f1, f2;
  const long long off = cell_offset(g, i, j, k, f0, f1, f2);
  const double v = W[(long long)c * g.ncell + off];
  return cell_flip(g, c, f0, f1, f2) ? -v : v;
}

// time of the prescribed states in stage STAGE of a step of length dt
// (stage 2 works on W*, the state at the half step)
__device__ __forceinline__ double boundary_time(const StageArgs& a, int stage, double dt) {
#pragma clang fp contract(off)
  if (!a.pb.on) return 0.0;
  const double t = a.t0 + (a.tclk ? *a.tclk : 0.0);
  return stage == 2 ? t + 0.5 * dt : t;
}

// load_cell with prescribed sides resolved first (x side, then y side): the
// given state at the ghost cell's centre, or the far kind's image
__device__ __forceinline__ double cell_value(const Geom& g, const Prescribed& pb, const double* W, int c, int i,
                                             int j, double tb) {
#pragma clang fp contract(off)
  if (!pb.on) return load_cell(g, W, c, i, j, 0);
  int lo0 = g.bclo[0], hi0 = g.bchi[0], lo1 = g.bclo[1], hi1 = g.bchi[1];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if (d >= g.D) break;
    const int id = d == 0 ? i : j;
    const int n = g.n[d];
    if (id >= 0 && id < n) continue;
    const bool low = id < 0;
    const int kind = d == 0 ? (low ? lo0 : hi0) : (low ? lo1 : hi1);
    if (kind != BC_PRESCRIBED) continue;
    const double s = g.D == 2 ? ((double)(d == 0 ? j : i) + 0.5) * g.dx[1 - d] : 0.0;
    const double r = ((double)id + 0.5) * g.dx[d];
    const double* L = low ? pb.line[d][0] : pb.line[d][1];
    if (s < (L[0] + L[1] * r) + L[2] * tb) return pb.A[c];
    const int far = low ? pb.far[d][0] : pb.far[d][1];
    if (far == BC_PRESCRIBED) return pb.B[c];
    if (d == 0) {
      if (low) lo0 = far; else hi0 = far;
    } else {
      if (low) lo1 = far; else hi1 = far;
    }
  }
  int f0 = 0, f1 = 0;
  const int ii = map_index(i, g.n[0], lo0, hi0, f0);
  const int jj = g.D >= 2 ? map_index(j, g.n[1], lo1, hi1, f1) : 0;
  double v = W[(long long)c * g.ncell + (long long)jj * g.n[0] + ii];
  if (c >= 1 && c <= g.D) {
    const int fo = c == 1 ? f0 : f1;
    if ((fo == 1) ^ (f0 == 2) ^ (f1 == 2)) v = -v;
  }
  return v;
}

// density and pressure of a frame-ordered Gauss-point state positive and
// finite, in one fixed operation order (the fallback's test)
template <int NC>
__device__ __forceinline__ bool physical_state(const double* w, double gamma) {
#pragma clang fp contract(off)
  double ke = 0.0;
#pragma unroll
  for (int q = 1; q < NC - 1; ++q) ke = ke + w[q] * w[q];
  const double pr = (gamma - 1.0) * (w[NC - 1] - 0.5 * ke / w[0]);
  return w[0] > 0.0 && pr > 0.0 && isfinite(w[0]) && isfinite(pr);
}

// first-order fallback: a non-physical side state becomes the side's cell
// average C with zero slopes; returns 1 if it did
template <int NC, int ND>
__device__ __forceinline__ int fallback_side(double* w, double (*dw)[NC], const double* C, double gamma) {
  if (physical_state<NC>(w, gamma)) return 0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    w[q] = C[q];
#pragma unroll
    for (int d = 0; d < ND; ++d) dw[d][q] = 0.0;
  }
  return 1;
}

template <int NC>
__device__ __forceinline__ void write_combined(int STAGE, const double* Fdt, const double* Fh, double w,
                                               double* accA, double* accB) {
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    if (STAGE == 1) {
      accA[q] += w * Fh[q];
      accB[q] += w * ((8.0 / 3.0) * Fh[q] - (1.0 / 3.0) * Fdt[q]);
    } else {
      accA[q] += w * ((4.0 / 3.0) * Fdt[q] - (8.0 / 3.0) * Fh[q]);
    }
  }
}

// A no-slip adiabatic wall is impermeable and, at rest, does no work and
// conducts no heat: the mass and energy fluxes of its faces are zero (frame
// components 0 and NC-1); f: face index along the normal axis ax.
template <int NC>
__device__ __forceinline__ void wall_fluxes(const Geom& g, int ax, int f, double* accA, double* accB) {
  if ((f == 0 && g.bclo[ax] == BC_NOSLIP) || (f == g.n[ax] && g.bchi[ax] == BC_NOSLIP)) {
    accA[0] = accA[NC - 1] = 0.0;
    accB[0] = accB[NC - 1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 1-D: one thread per face.
// ---------------------------------------------------------------------------
// EX: prescribed sides or the first-order fallback may be on (a separate
// instantiation, so that grids without them run the plain code)
// SCHEME: the reconstruction (SCHEME_TENO_D, the paper's scheme, or one of
// its comparison schemes)
template <int STAGE, bool NS, bool FLAGS, bool CHAR = false, bool EX = false, int SCHEME = SCHEME_TENO_D>
__device__ __forceinline__ void face1d_body(const StageArgs& a, int f) {
  const double dt = *a.dt;
  if (!(dt > 0.0)) return;
  const int n = a.g.n[0];
  if (f > n) return;
  double Wl[3], Wr[3], dWl[1][3], dWr[1][3], dW0[1][3];
  const double idx = 1.0 / a.g.dx[0];  // normal slopes per unit length
  const double tb = EX ? boundary_time(a, STAGE, dt) : 0.0;
  if (CHAR) {
    double C[6][3];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        C[r][c] = EX ? cell_value(a.g, a.pb, a.W, c, f - 3 + r, 0, tb) : load_cell(a.g, a.W, c, f - 3 + r, 0, 0);
    unsigned fr[3];
    char_recon_face<1>(a.gamma, C, a.tn, idx, Wl, dWl[0], Wr, dWr[0], fr);
    if (FLAGS && f < n)
#pragma unroll
      for (int k = 0; k < 3; ++k) a.nflags[(long long)k * n + f] = (uint8_t)fr[k];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double Q[6];
#pragma unroll
      for (int r = 0; r < 6; ++r)
        Q[r] = EX ? cell_value(a.g, a.pb, a.W, c, f - 3 + r, 0, tb) : load_cell(a.g, a.W, c, f - 3 + r, 0, 0);
      double o[4];
      if (SCHEME == SCHEME_TENO_D) {
        const unsigned fl = teno_flag<SEL_FILTER>(Q, a.tn);
        teno_face(Q, fl, o);
        Wl[c] = o[2];
        dWl[0][c] = o[3] * idx;
        const unsigned fr = teno_flag<SEL_FILTER>(Q + 1, a.tn);
        teno_face(Q + 1, fr, o);
        Wr[c] = o[0];
        dWr[0][c] = o[1] * idx;
        if (FLAGS && f < n) a.nflags[(long long)c * n + f] = (uint8_t)fr;
      } else {
        scheme_face<SCHEME>(Q, a.sc, o);
        Wl[c] = o[2];
        dWl[0][c] = o[3] * idx;
        const unsigned fr = scheme_face<SCHEME>(Q + 1, a.sc, o);
        Wr[c] = o[0];
        dWr[0][c] = o[1] * idx;
        if (FLAGS && f < n) a.nflags[(long long)c * n + f] = (uint8_t)fr;
        // separately reconstructed equilibrium slope (Eq. 3.12)
        if (SCHEME >= SCHEME_TENO5) dW0[0][c] = eq_slope(Q[1], Q[2], Q[3], Q[4]) * idx;
      }
    }
  }
  if (EX && a.fallback) {
    double Cl[3], Cr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Cl[c] = cell_value(a.g, a.pb, a.W, c, f - 1, 0, tb);
      Cr[c] = cell_value(a.g, a.pb, a.W, c, f, 0, tb);
    }
    const int nfb = fallback_side<3, 1>(Wl, dWl, Cl, a.gamma) + fallback_side<3, 1>(Wr, dWr, Cr, a.gamma);
    if (nfb && a.fbc) atomicAdd(a.fbc, (unsigned long long)nfb);
  }
  double Fdt[3], Fh[3], A[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  const bool ok = SCHEME >= SCHEME_TENO5
                      ? gp_flux_eq<1, NS>(Wl, Wr, dWl, dWr, (const double*)nullptr, dW0, a.fc, dt, Fdt, Fh)
                      : gp_flux<1, NS>(Wl, Wr, dWl, dWr, a.fc, dt, Fdt, Fh);
  if (!ok) atomicAdd(a.fail, 1ull);
  write_combined<3>(STAGE, Fdt, Fh, 1.0, A, B);
  wall_fluxes<3>(a.g, 0, f, A, B);
  const long long nf = n + 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.FA[c * nf + f] = A[c];
    if (STAGE == 1) a.FB[c * nf + f] = B[c];
  }
}

template <int STAGE, bool NS, bool FLAGS, bool CHAR = false, bool EX = false, int SCHEME = SCHEME_TENO_D>
__global__ __launch_bounds__(256) void face1d_kernel(StageArgs a) {
  face1d_body<STAGE, NS, FLAGS, CHAR, EX, SCHEME>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// 2-D: fused face kernel.  A block owns TN faces along the normal axis AX by
// TT rows along the tangential axis.  It stages the cells of the tile with a
// halo of 3 (normal) and 2 (tangential) in LDS, reconstructs every needed
// cell once along AX into LDS (values and normal slopes on both faces), and
// then each thread reconstructs its face's left and right states along the
// face at the two Gauss points and evaluates the two Gauss-point fluxes.
// ---------------------------------------------------------------------------
// Tile shapes (faces along the normal x faces along the tangential axis),
// two lanes per face; chosen per grid by the autotuner.
constexpr int NTILE2 = 3;
constexpr int CHAR_TILE2 = 2;  // the one tile shape of the characteristic path
__host__ __device__ constexpr int tile2_tn(int k) { return k == 0 ? 16 : (k == 1 ? 16 : 8); }
__host__ __device__ constexpr int tile2_tt(int k) { return k == 0 ? 8 : (k == 1 ? 16 : 16); }

// LDS doubles of one 2-D face tile: the staged cells and their normal
// reconstruction
__host__ __device__ constexpr int tile2_lds(int k) {
  return 4 * (tile2_tt(k) + 4) * (tile2_tn(k) + 5) + 4 * (tile2_tt(k) + 4) * (tile2_tn(k) + 1) * 4;
}

// ... plus, with characteristic variables, the per-face field values of both
// sides and the right eigenvectors of every staged face row
__host__ __device__ constexpr int tile2_lds_char(int k) {
  return tile2_lds(k) + 4 * (tile2_tt(k) + 4) * tile2_tn(k) * 4 + (tile2_tt(k) + 4) * tile2_tn(k) * 16;
}

// ... plus, with a separately reconstructed equilibrium (WENO-Z, TENO5),
// the equilibrium state and its normal slope of every staged face segment
__host__ __device__ constexpr int tile2_lds_eq(int k) {
  return tile2_lds(k) + 2 * 4 * (tile2_tt(k) + 4) * tile2_tn(k);
}

// (bx, by): tile index along the normal and the tangential axis; lds: the
// block's tile2_lds(TILE) (CHAR: tile2_lds_char(TILE); SCHEME_TENO5 and
// SCHEME_WENO_Z: tile2_lds_eq(TILE)) doubles of shared memory.  CHAR:
// reconstruction in characteristic variables (steps 2 and 3 below project
// onto the fields of each face and back).  SCHEME: the reconstruction
// (SCHEME_TENO_D or a comparison scheme; conservative variables).
template <int AX, int STAGE, bool NS, bool FLAGS, int TILE, bool CHAR = false, bool EX = false,
          int SCHEME = SCHEME_TENO_D>
__device__ __forceinline__ void face2d_tile(const StageArgs& a, int bx, int by, double* lds) {
  constexpr int TN = tile2_tn(TILE), TT = tile2_tt(TILE), NT = 2 * TN * TT;
  constexpr int NC = 4;
  constexpr int LN = TN + 5, LT = TT + 4, RN = TN + 1;
  double(*sW)[LT][LN] = reinterpret_cast<double(*)[LT][LN]>(lds);
  double(*sR)[LT][RN][4] = reinterpret_cast<double(*)[LT][RN][4]>(lds + NC * LT * LN);
  const double dt = *a.dt;
  if (!(dt > 0.0)) return;
  const Geom& g = a.g;
  const int TA = 1 - AX;  // tangential axis
  const int nN = g.n[AX], nT = g.n[TA];
  const int f0 = bx * TN, t0 = by * TT;
  const int tid = threadIdx.x;
  const double tb = EX ? boundary_time(a, STAGE, dt) : 0.0;

  // 1. cells of the tile, ghost cells by the index map or prescribed states;
  //    without prescribed sides one thread per cell maps it once and loads
  //    its four components
  if (EX) {
    for (int L = tid; L < NC * LN * LT; L += NT) {
      int nl, tl;
      if (AX == 0) {
        nl = L % LN;
        tl = (L / LN) % LT;
      } else {
        tl = L % LT;
        nl = (L / LT) % LN;
      }
      const int c = L / (LN * LT);
      const int pn = f0 - 3 + nl, pt = t0 - 2 + tl;
      sW[c][tl][nl] = cell_value(g, a.pb, a.W, c, AX == 0 ? pn : pt, AX == 0 ? pt : pn, tb);
    }
  } else {
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
  }
  __syncthreads();

  // 2. normal reconstruction of cells f0-1 .. f0+TN-1 on every staged row
  const double idn = 1.0 / g.dx[AX];  // normal slopes per unit length
  const int perm[NC] = {0, 1 + AX, 1 + TA, 3};
  if (CHAR) {
    // per face and row: the fields of the face's normal basis.  (a) one
    // thread per (side, row, face) projects the side's five cells, selects
    // and reconstructs every field; the left-side thread also keeps the
    // right eigenvectors.  (b) one thread per (component, row, face) projects
    // back.  Same slots of sR as the conservative path: face fn's left state
    // in cell slot fn (high face), its right state in slot fn + 1 (low face).
    double(*sV)[LT][TN][4] = reinterpret_cast<double(*)[LT][TN][4]>(lds + tile2_lds(TILE));
    double(*sM)[TN][16] = reinterpret_cast<double(*)[TN][16]>(lds + tile2_lds(TILE) + NC * LT * TN * 4);
    for (int L = tid; L < 2 * LT * TN; L += NT) {
      const int fn = L % TN;
      const int tl = (L / TN) % LT;
      const int sd = L / (TN * LT);
      double C[6][NC];
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int q = 0; q < NC; ++q) C[r][q] = sW[perm[q]][tl][fn + r];
      double Wb[NC], Lm[NC][NC], Rm[NC][NC];
      {
#pragma clang fp contract(off)
#pragma unroll
        for (int q = 0; q < NC; ++q) Wb[q] = 0.5 * (C[2][q] + C[3][q]);
      }
      char_basis<2, 0>(a.gamma, Wb, Lm, Rm);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        double V[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) V[r] = char_dot<NC>(Lm[k], sd == 0 ? C[r] : C[r + 1]);
        const unsigned fl = teno_flag<SEL_FILTER>(V, a.tn);
        double o[4];
        teno_face(V, fl, o);
        if (sd == 0) {
          sV[k][tl][fn][0] = o[2];
          sV[k][tl][fn][1] = o[3];
        } else {
          sV[k][tl][fn][2] = o[0];
          sV[k][tl][fn][3] = o[1];
          if (FLAGS) {
            const int cell = f0 + fn, row = t0 - 2 + tl;
            if (cell < nN && tl >= 2 && tl < TT + 2 && row < nT) {
              const long long lin = AX == 0 ? (long long)row * g.n[0] + cell : (long long)cell * g.n[0] + row;
              a.nflags[((long long)AX * NC + k) * g.ncell + lin] = (uint8_t)fl;
            }
          }
        }
      }
      if (sd == 0)
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
          for (int k = 0; k < NC; ++k) sM[tl][fn][q * NC + k] = Rm[q][k];
    }
    __syncthreads();
    for (int L = tid; L < NC * LT * TN; L += NT) {
      const int fn = L % TN;
      const int tl = (L / TN) % LT;
      const int q = L / (TN * LT);
      const double* rq = &sM[tl][fn][q * NC];
      double x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double v[NC] = {sV[0][tl][fn][j], sV[1][tl][fn][j], sV[2][tl][fn][j], sV[3][tl][fn][j]};
        x[j] = char_dot<NC>(rq, v);
      }
      const int c = q == 0 ? perm[0] : (q == 1 ? perm[1] : (q == 2 ? perm[2] : perm[3]));
      sR[c][tl][fn][2] = x[0];
      sR[c][tl][fn][3] = x[1] * idn;
      sR[c][tl][fn + 1][0] = x[2];
      sR[c][tl][fn + 1][1] = x[3] * idn;
    }
  } else {
    for (int L = tid; L < NC * LT * RN; L += NT) {
      const int nr = L % RN;
      const int tl = (L / RN) % LT;
      const int c = L / (RN * LT);
      const double* Q = &sW[c][tl][nr];
      double o[4];
      unsigned fl;
      if (SCHEME == SCHEME_TENO_D) {
        fl = teno_flag<SEL_FILTER>(Q, a.tn);
        teno_face(Q, fl, o);
      } else {
        fl = scheme_face<SCHEME>(Q, a.sc, o);
      }
      sR[c][tl][nr][0] = o[0];
      sR[c][tl][nr][1] = o[1] * idn;
      sR[c][tl][nr][2] = o[2];
      sR[c][tl][nr][3] = o[3] * idn;
      if (FLAGS) {
        const int cell = f0 - 1 + nr, row = t0 - 2 + tl;
        if (nr >= 1 && cell < nN && tl >= 2 && tl < TT + 2 && row < nT) {
          const long long lin = AX == 0 ? (long long)row * g.n[0] + cell : (long long)cell * g.n[0] + row;
          a.nflags[((long long)AX * NC + c) * g.ncell + lin] = (uint8_t)fl;
        }
      }
    }
  }
  __syncthreads();

  // 2b. WENO-Z / TENO5: the equilibrium state of every staged face segment,
  //     the kinetic weighting of its two line-averaged interface states
  //     (Eq. 2.6), and its normal slope from the cells (Eq. 3.12), frame
  //     order; reconstructed along the face at the Gauss points in step 3
  double(*sE)[2][LT][TN] = reinterpret_cast<double(*)[2][LT][TN]>(lds + tile2_lds(TILE));
  if (SCHEME >= SCHEME_TENO5) {
    for (int L = tid; L < LT * TN; L += NT) {
      const int fn = L % TN, tl = L / TN;
      double wl[NC], wr[NC], sl[NC], sr[NC], h0, h1, k0, k1;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        wl[q] = sR[perm[q]][tl][fn][2];
        wr[q] = sR[perm[q]][tl][fn + 1][0];
      }
      Gas<2, double> gl, gr;
      side_w0<2>(wl, a.fc, 1.0, gl, h0, h1, sl);
      side_w0<2>(wr, a.fc, -1.0, gr, k0, k1, sr);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int c = perm[q];
        sE[q][0][tl][fn] = sl[q] + sr[q];
        sE[q][1][tl][fn] = eq_slope(sW[c][tl][fn + 1], sW[c][tl][fn + 2], sW[c][tl][fn + 3], sW[c][tl][fn + 4]) * idn;
      }
    }
    __syncthreads();
  }

  // 3. lanes 2k and 2k+1 share face k.  Lane m reconstructs side m (left: 0,
  //    right: 1) along the face at both Gauss points, keeps Gauss point m and
  //    hands Gauss point 1-m to its partner; each lane then evaluates the
  //    flux at its Gauss point m and the pair sums the two.
  const int m = tid & 1;
  const int fi = tid >> 1;
  const int fn = fi % TN, ft = fi / TN;
  const int f = f0 + fn, t = t0 + ft;
  const bool live = f <= nN && t < nT;
  const long long nf = face_count(g, AX);
  const long long fidx = AX == 0 ? (long long)t * (g.n[0] + 1) + f : (long long)f * g.n[0] + t;
  const double idt = 1.0 / g.dx[TA];
  double Wg[2][NC], Dg[2][2][NC];  // [side][q], [side][axis n/t][q]
  const int nr = m == 0 ? fn : fn + 1;
  const int vo = m == 0 ? 2 : 0;
  if (CHAR) {
    // fields of the basis along the face at this face's reference state
    // (cells f-1 and f of row t); each field of W and of W_n is selected and
    // evaluated at both Gauss points, then projected back
    double aV[NC][2], aD[NC][2], aN[NC][2];
#pragma unroll
    for (int q = 0; q < NC; ++q) aV[q][0] = aV[q][1] = aD[q][0] = aD[q][1] = aN[q][0] = aN[q][1] = 0.0;
    if (live) {
      double Wb[NC], Lt[NC][NC], Rt[NC][NC];
      {
#pragma clang fp contract(off)
#pragma unroll
        for (int q = 0; q < NC; ++q) Wb[q] = 0.5 * (sW[perm[q]][ft + 2][fn + 2] + sW[perm[q]][ft + 2][fn + 3]);
      }
      char_basis<2, 1>(a.gamma, Wb, Lt, Rt);
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        double Qw[5], Qn[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
          double xw[NC], xn[NC];
#pragma unroll
          for (int q = 0; q < NC; ++q) {
            xw[q] = sR[perm[q]][ft + r][nr][vo];
            xn[q] = sR[perm[q]][ft + r][nr][vo + 1];
          }
          Qw[r] = char_dot<NC>(Lt[k], xw);
          Qn[r] = char_dot<NC>(Lt[k], xn);
        }
        const unsigned fw = teno_flag<SEL_FILTER>(Qw, a.tt);
        const unsigned fq = teno_flag<SEL_FILTER>(Qn, a.tt);
        if (FLAGS) {
          a.tflags[((long long)(0 * 2 + m) * NC + k) * nf + fidx] = (uint8_t)fw;
          a.tflags[((long long)(1 * 2 + m) * NC + k) * nf + fidx] = (uint8_t)fq;
        }
        double v[2], dv[2], vn[2], dvn[2];
        teno_gauss(Qw, fw, v, dv);
        teno_gauss(Qn, fq, vn, dvn);
        {
          // back-projection: dense sums in field order, no contraction
#pragma clang fp contract(off)
#pragma unroll
          for (int q = 0; q < NC; ++q)
#pragma unroll
            for (int gp = 0; gp < 2; ++gp) {
              aV[q][gp] = aV[q][gp] + Rt[q][k] * v[gp];
              aD[q][gp] = aD[q][gp] + Rt[q][k] * dv[gp];
              aN[q][gp] = aN[q][gp] + Rt[q][k] * vn[gp];
            }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      // selects, not an index by the lane's m (which would place the
      // arrays in scratch memory)
      const double sv = m ? aV[q][0] : aV[q][1], sd = m ? aD[q][0] : aD[q][1], sn = m ? aN[q][0] : aN[q][1];
      const double rv = lane_xor<1>(sv), rd = lane_xor<1>(sd), rn = lane_xor<1>(sn);
      const double ov = m ? aV[q][1] : aV[q][0], od = m ? aD[q][1] : aD[q][0], on = m ? aN[q][1] : aN[q][0];
      Wg[0][q] = m == 0 ? ov : rv;
      Wg[1][q] = m == 0 ? rv : ov;
      Dg[0][1][q] = (m == 0 ? od : rd) * idt;
      Dg[1][1][q] = (m == 0 ? rd : od) * idt;
      Dg[0][0][q] = m == 0 ? on : rn;
      Dg[1][0][q] = m == 0 ? rn : on;
    }
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = perm[q];
      double v[2] = {0, 0}, dv[2] = {0, 0}, vn[2] = {0, 0}, dvn[2];
      if (live) {
        double Qw[5], Qn[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
          Qw[r] = sR[c][ft + r][nr][vo];
          Qn[r] = sR[c][ft + r][nr][vo + 1];
        }
        unsigned fw, fq;
        if (SCHEME == SCHEME_TENO_D) {
          fw = teno_flag<SEL_FILTER>(Qw, a.tt);
          fq = teno_flag<SEL_FILTER>(Qn, a.tt);
          teno_gauss(Qw, fw, v, dv);
          teno_gauss(Qn, fq, vn, dvn);
        } else {
          fw = scheme_gauss<SCHEME>(Qw, a.sc, v, dv);
          fq = scheme_gauss<SCHEME>(Qn, a.sc, vn, dvn);
        }
        if (FLAGS) {
          a.tflags[((long long)(0 * 2 + m) * NC + c) * nf + fidx] = (uint8_t)fw;
          a.tflags[((long long)(1 * 2 + m) * NC + c) * nf + fidx] = (uint8_t)fq;
        }
      }
      // own side at own Gauss point; the partner's side at this Gauss point
      // arrives from the partner, which computed it
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
  double A[NC] = {0, 0, 0, 0}, B[NC] = {0, 0, 0, 0};
  if (EX && live && a.fallback) {
    double Cl[NC], Cr[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      Cl[q] = sW[perm[q]][ft + 2][fn + 2];
      Cr[q] = sW[perm[q]][ft + 2][fn + 3];
    }
    const int nfb = fallback_side<NC, 2>(Wg[0], Dg[0], Cl, a.gamma) + fallback_side<NC, 2>(Wg[1], Dg[1], Cr, a.gamma);
    if (nfb && a.fbc) atomicAdd(a.fbc, (unsigned long long)nfb);
  }
  if (live) {
    double Fdt[NC], Fh[NC];
    bool ok;
    if (SCHEME >= SCHEME_TENO5) {
      // the equilibrium at this lane's Gauss point: the five face segments'
      // states reconstructed with the cut-off of Sec. 4.1 (TENO5, q = 6;
      // the linear quartic where they are smooth, Sec. 3.1 Step 4), value
      // and derivatives
      SchemeCfg se = a.sc;
      se.q = 6;
      double W0e[NC], dW0e[2][NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        double Qe[5], Qx[5], v[2], d[2];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
          Qe[r] = sE[q][0][ft + r][fn];
          Qx[r] = sE[q][1][ft + r][fn];
        }
        scheme_gauss<SCHEME_TENO5>(Qe, se, v, d);
        W0e[q] = m ? v[1] : v[0];
        dW0e[1][q] = (m ? d[1] : d[0]) * idt;
        scheme_gauss<SCHEME_TENO5>(Qx, se, v, d);
        dW0e[0][q] = m ? v[1] : v[0];
      }
      ok = gp_flux_eq<2, NS>(Wg[0], Wg[1], Dg[0], Dg[1], W0e, dW0e, a.fc, dt, Fdt, Fh);
    } else {
      ok = gp_flux<2, NS>(Wg[0], Wg[1], Dg[0], Dg[1], a.fc, dt, Fdt, Fh);
    }
    if (!ok) atomicAdd(a.fail, 1ull);
    write_combined<NC>(STAGE, Fdt, Fh, 0.5, A, B);
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    A[q] += lane_xor<1>(A[q]);
    if (STAGE == 1) B[q] += lane_xor<1>(B[q]);
  }
  wall_fluxes<NC>(g, AX, f, A, B);
  if (live && m == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      a.FA[(long long)perm[q] * nf + fidx] = A[q];
      if (STAGE == 1) a.FB[(long long)perm[q] * nf + fidx] = B[q];
    }
  }
}

template <int AX, int STAGE, bool NS, bool FLAGS, int TILE>
__global__ __launch_bounds__(2 * tile2_tn(TILE) * tile2_tt(TILE), 2) void face2d_kernel(StageArgs a) {
  __shared__ double lds[tile2_lds(TILE)];
  face2d_tile<AX, STAGE, NS, FLAGS, TILE>(a, blockIdx.x, blockIdx.y, lds);
}

// Both directions in one launch: the first blocks take the x-face tiles,
// the rest the y-face tiles (one shared LDS tile), so that neither
// direction waits for the other's tail.
template <int STAGE, bool NS, bool FLAGS, int TILE, bool CHAR = false, bool EX = false, int SCHEME = SCHEME_TENO_D>
__global__ __launch_bounds__(2 * tile2_tn(TILE) * tile2_tt(TILE), 2) void face2d_xy_kernel(StageArgs ax,
                                                                                           StageArgs ay) {
  constexpr int TN = tile2_tn(TILE);
  __shared__ double lds[CHAR ? tile2_lds_char(TILE) : (SCHEME >= SCHEME_TENO5 ? tile2_lds_eq(TILE) : tile2_lds(TILE))];
  const int nbx = (ax.g.n[0] + 1 + TN - 1) / TN;          // x faces: tiles along x
  const int nx = nbx * ((ax.g.n[1] + tile2_tt(TILE) - 1) / tile2_tt(TILE));
  // XCD-aware order: workgroups are dealt to the 8 XCDs in turn; the tiles
  // are renumbered so that each XCD walks a contiguous range of them (a
  // bijection for any grid size), where neighbouring tiles, which stage
  // common halo cells and write common cache lines of the face fluxes,
  // meet in one L2 (HBM reads per launch fall 2.7-3.0x, writes to the
  // algorithmic bytes).
  const int nbt = gridDim.x, x8 = blockIdx.x & 7, per = nbt >> 3, rem = nbt & 7;
  const int b = x8 * per + min(x8, rem) + (int)(blockIdx.x >> 3);
  if (b < nx) {
    face2d_tile<0, STAGE, NS, FLAGS, TILE, CHAR, EX, SCHEME>(ax, b % nbx, b / nbx, lds);
  } else {
    const int nby = (ay.g.n[1] + 1 + TN - 1) / TN;        // y faces: tiles along y
    face2d_tile<1, STAGE, NS, FLAGS, TILE, CHAR, EX, SCHEME>(ay, (b - nx) % nby, (b - nx) / nby, lds);
  }
}

// ---------------------------------------------------------------------------
// 3-D.  (a) normal reconstruction along AX of every cell with AX index in
// [-1, n] (interior in the other axes): R[c][4][k][j][i'] with the AX index
// shifted by one, values and slopes on both faces.
// ---------------------------------------------------------------------------
template <int AX, bool FLAGS>
__global__ __launch_bounds__(256) void recon3d_kernel(StageArgs a) {
  const Geom& g = a.g;
  int ext[3] = {g.n[0], g.n[1], g.n[2]};
  ext[AX] += 2;
  const long long nr = (long long)ext[0] * ext[1] * ext[2];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nr * 5) return;
  const int c = (int)(id / nr);
  long long r = id % nr;
  int p[3];
  p[0] = (int)(r % ext[0]);
  r /= ext[0];
  p[1] = (int)(r % ext[1]);
  p[2] = (int)(r / ext[1]);
  p[AX] -= 1;
  // the stencil runs along AX only (the other indices are interior): one
  // base offset, and the index map along AX for each of its five cells
  const long long sax = AX == 0 ? 1 : (AX == 1 ? (long long)g.n[0] : (long long)g.n[0] * g.n[1]);
  int pz[3] = {p[0], p[1], p[2]};
  pz[AX] = 0;
  const double* Wc = a.W + (long long)c * g.ncell + ((long long)pz[2] * g.n[1] + pz[1]) * g.n[0] + pz[0];
  double Q[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    int f[3] = {0, 0, 0};
    const int m = map_index(p[AX] + s - 2, g.n[AX], g.bclo[AX], g.bchi[AX], f[AX]);
    const double v = Wc[m * sax];
    Q[s] = cell_flip(g, c, f[0], f[1], f[2]) ? -v : v;
  }
  const unsigned fl = teno_flag<SEL_RATIO>(Q, a.tn);
  double o[4];
  teno_face(Q, fl, o);
  const double idn = 1.0 / g.dx[AX];
  const long long base = (long long)c * 4 * nr + (id % nr);
  a.Rout[base] = o[0];
  a.Rout[base + nr] = o[1] * idn;
  a.Rout[base + 2 * nr] = o[2];
  a.Rout[base + 3 * nr] = o[3] * idn;
  if (FLAGS && p[AX] >= 0 && p[AX] < g.n[AX])
    a.nflags[((long long)AX * 5 + c) * g.ncell + ((long long)p[2] * g.n[1] + p[1]) * g.n[0] + p[0]] = (uint8_t)fl;
}

// (b) face kernel.  A block owns one plane of faces (fixed index along AX)
// and a B1 x B2 tile of it along the tangential axes T1, T2 (cyclic order:
// x-faces y, z; y-faces z, x; z-faces x, y).  It stages the normal
// reconstruction of both sides (from recon3d_kernel) with a halo of two in
// LDS (ghost positions by the index map, mirrored momenta negated),
// reconstructs every face line of the tile and its T2 halo once along T1
// (sweep 1, both T1 Gauss points), and then eight lanes share a face: lane
// (m1, m3, m2) owns side m2 at Gauss point (m1, m3).
//   * Sweep 2: the pair (m3 = 0, 1) of a side and T1 point splits the
//     fifteen T2 reconstructions of that side (five components of the value,
//     its T1 derivative and its normal slope) and swaps the results at each
//     other's T2 point.
//   * Flux: each lane evaluates its side's share of the equilibrium state
//     and of the non-equilibrium moments (side_w0, side_part); the pair
//     (m2 = 0, 1) adds the shares (a + b is exact-order independent), and
//     both lanes evaluate the equilibrium part (flux_combine).  One side per
//     lane keeps the flux within the register budget of two waves per SIMD.
// Tiles are dealt to the 8 XCDs in contiguous ranges.
// FLAGS: record the tangential selections (stage 1), per face of this
// direction: sweep 1 of the face's own line as [(q*2 + side)*5 + c] (q = 0:
// W, 1: W_n), then sweep 2 as [20 + ((m1*3 + kind)*2 + side)*5 + c] (kind 0:
// W, 1: dW/dt1, 2: W_n at T1 Gauss point m1), c the global component, each a
// plane of faces indexed like a state whose axis AX has n + 1 entries.
constexpr int B3_1 = 2, B3_2 = 16, L3 = 8;

template <int AX, int STAGE, bool NS, bool EX = false, bool FLAGS = false>
__global__ __launch_bounds__(L3 * B3_1 * B3_2, 2) void face3d_kernel(StageArgs a) {
  constexpr int NC = 5, B1 = B3_1, B2 = B3_2, NT = L3 * B1 * B2;
  constexpr int L1 = B1 + 4, L2 = B2 + 4;
  constexpr int T1 = (AX + 1) % 3, T2 = (AX + 2) % 3;
  __shared__ double sR[2][NC][2][L2][L1];      // [side][c][value, normal slope][t2][t1]
  __shared__ double sS[2][NC][L2][B1][6];      // sweep 1: v(m1), d_t1 v(m1), v_n(m1)
  const double dt = *a.dt;
  if (!(dt > 0.0)) return;
  const Geom& g = a.g;
  // XCD-aware order: workgroups are dealt to the 8 XCDs in turn; the
  // logical tiles are renumbered so that each XCD walks a contiguous range
  // in which tiles that share cache lines of the normal reconstruction
  // (x fastest in memory) follow each other and meet in one L2: for the
  // x faces the face plane is fastest (neighbouring planes share the lines
  // along x), for the y and z faces the T1 tile (the z-rows of the y faces'
  // tiles overlap by four of six, the z faces' tiles cover the x-lines two
  // cells at a time), then the plane, then the T2 tile.
  const int nb1 = (g.n[T1] + B1 - 1) / B1, nb2 = (g.n[T2] + B2 - 1) / B2;
  const int np = g.n[AX] + 1;
  const int nbl = np * nb1 * nb2;
  const int per = (nbl + 7) / 8;
  const int lb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lb >= nbl) return;
  const int fa = AX == 0 ? lb % np : (lb / nb1) % np;
  const int t10 = (AX == 0 ? (lb / np) % nb1 : lb % nb1) * B1, t20 = (lb / (np * nb1)) * B2;
  const int tid = threadIdx.x;
  int ext[3] = {g.n[0], g.n[1], g.n[2]};
  ext[AX] += 2;
  const long long nr = (long long)ext[0] * ext[1] * ext[2];

  // 1. normal reconstruction of the two cells beside each face position:
  //    thread (position, k) maps its tangential position once and loads
  //    both sides' five components of the value (k = 0) or the normal slope
  //    (k = 1); x, the fastest axis in memory, runs fastest over threads
  static_assert(2 * L1 * L2 <= NT, "one thread per position and kind");
  if (tid < 2 * L1 * L2) {
    const int p = tid % (L1 * L2), k = tid / (L1 * L2);
    const int i1 = AX == 1 ? p / L2 : p % L1;
    const int i2 = AX == 1 ? p % L2 : p / L1;
    int f1 = 0, f2 = 0;
    int e[3];
    e[AX] = fa;  // cell fa - 1 along AX, shifted by one; the right side is the next
    e[T1] = map_index(t10 - 2 + i1, g.n[T1], g.bclo[T1], g.bchi[T1], f1);
    e[T2] = map_index(t20 - 2 + i2, g.n[T2], g.bclo[T2], g.bchi[T2], f2);
    const long long off = ((long long)e[2] * ext[1] + e[1]) * ext[0] + e[0];
    const long long sax = AX == 0 ? 1 : (AX == 1 ? (long long)ext[0] : (long long)ext[0] * ext[1]);
    double v[2][NC];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < NC; ++c) v[s][c] = a.R[(long long)(c * 4 + (s == 0 ? 2 : 0) + k) * nr + off + s * sax];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const bool mom = c >= 1 && c <= 3;
      const bool neg = (c == 1 + T1 && f1 == 1) ^ (c == 1 + T2 && f2 == 1) ^ (mom && f1 == 2) ^ (mom && f2 == 2);
#pragma unroll
      for (int s = 0; s < 2; ++s) sR[s][c][k][i2][i1] = neg ? -v[s][c] : v[s][c];
    }
  }
  __syncthreads();

  // 2. sweep 1 along T1 of every face line of the tile and its T2 halo
  const double i1d = 1.0 / g.dx[T1], i2d = 1.0 / g.dx[T2];
  int nfa[3] = {g.n[0], g.n[1], g.n[2]};
  nfa[AX] += 1;
  const long long nf = (long long)nfa[0] * nfa[1] * nfa[2];
  for (int L = tid; L < 2 * NC * L2 * B1; L += NT) {
    const int j1 = L % B1;
    const int i2 = (L / B1) % L2;
    const int c = (L / (B1 * L2)) % NC;
    const int s = L / (NC * B1 * L2);
    double Qw[5], Qn[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      Qw[r] = sR[s][c][0][i2][j1 + r];
      Qn[r] = sR[s][c][1][i2][j1 + r];
    }
    double v[2], dv[2], vn[2], dvn[2];
    const unsigned fw = teno_flag<SEL_RATIO>(Qw, a.tt), fq = teno_flag<SEL_RATIO>(Qn, a.tt);
    // the inputs of the second sweep's selections: one fixed evaluation order
    teno_gauss_exact(Qw, fw, v, dv);
    teno_gauss_exact(Qn, fq, vn, dvn);
    if (FLAGS && i2 >= 2 && i2 < B2 + 2) {
      int q3[3];
      q3[AX] = fa;
      q3[T1] = t10 + j1;
      q3[T2] = t20 + i2 - 2;
      if (q3[T1] < g.n[T1] && q3[T2] < g.n[T2]) {
        const long long fid = ((long long)q3[2] * nfa[1] + q3[1]) * nfa[0] + q3[0];
        a.tflags[((long long)(0 * 2 + s) * NC + c) * nf + fid] = (uint8_t)fw;
        a.tflags[((long long)(1 * 2 + s) * NC + c) * nf + fid] = (uint8_t)fq;
      }
    }
    double* o = sS[s][c][i2][j1];
    o[0] = v[0];
    o[1] = v[1];
    o[2] = dv[0] * i1d;
    o[3] = dv[1] * i1d;
    o[4] = vn[0];
    o[5] = vn[1];
  }
  __syncthreads();

  // 3. sweep 2 along T2, split over the pair m3 = 0, 1.  Item it = 3 q + kind
  //    (kind 0: value, 1: T1 derivative, 2: normal slope of component perm[q]);
  //    in round r lane m3 reconstructs item 2 r + m3 at both T2 points and
  //    hands its partner the value (and T2 derivative) at the partner's point.
  const int m2 = tid & 1, m3 = (tid >> 1) & 1, m1 = (tid >> 2) & 1, fi = tid >> 3;
  const int j1 = fi % B1, j2 = fi / B1;
  int fp[3];
  fp[AX] = fa;
  fp[T1] = t10 + j1;
  fp[T2] = t20 + j2;
  const bool live = fp[T1] < g.n[T1] && fp[T2] < g.n[T2];
  const long long fid = ((long long)fp[2] * nfa[1] + fp[1]) * nfa[0] + fp[0];
  const int perm[NC] = {0, 1 + AX, 1 + T1, 1 + T2, 4};
  double item[15], item_d[15];  // at this lane's T2 point: value, T2 derivative (cell units)
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int it = 2 * r + m3;
    double v[2] = {0.0, 0.0}, d[2] = {0.0, 0.0};
    if (live && it < 15) {
      const int q = it / 3, kind = it - 3 * q;
      const int c = q == 0 ? perm[0] : q == 1 ? perm[1] : q == 2 ? perm[2] : q == 3 ? perm[3] : perm[4];
      double Q[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) Q[k] = sS[m2][c][j2 + k][j1][2 * kind + m1];
      const unsigned fl = teno_flag<SEL_RATIO>(Q, a.tt);
      teno_gauss(Q, fl, v, d);
      if (FLAGS) a.tflags[((long long)4 * NC + ((m1 * 3 + kind) * 2 + m2) * NC + c) * nf + fid] = (uint8_t)fl;
    }
    const double own = m3 ? v[1] : v[0], own_d = m3 ? d[1] : d[0];
    const double rcv = lane_xor<2>(m3 ? v[0] : v[1]), rcv_d = lane_xor<2>(m3 ? d[0] : d[1]);
    // item 2 r is lane m3 = 0's, item 2 r + 1 lane m3 = 1's
    item[2 * r] = m3 ? rcv : own;
    item_d[2 * r] = m3 ? rcv_d : own_d;
    if (2 * r + 1 < 15) {
      item[2 * r + 1] = m3 ? own : rcv;
      item_d[2 * r + 1] = m3 ? own_d : rcv_d;
    }
  }
  double Ws[NC], dWs[3][NC];  // this lane's side at its Gauss point, face frame
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    Ws[q] = item[3 * q];
    dWs[2][q] = item_d[3 * q] * i2d;
    dWs[1][q] = item[3 * q + 1];
    dWs[0][q] = item[3 * q + 2];
  }
  if (EX && live && a.fallback) {
    // first-order fallback: this side's cell (fa - 1 + m2 along AX), frame order
    int cp[3] = {fp[0], fp[1], fp[2]};
    cp[AX] = fa - 1 + m2;
    double C[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) C[q] = load_cell(g, a.W, perm[q], cp[0], cp[1], cp[2]);
    if (fallback_side<NC, 3>(Ws, dWs, C, a.gamma) && a.fbc) atomicAdd(a.fbc, 1ull);
  }

  // 4. the Gauss-point flux, one side per lane
  Gas<3, double> gs, g0;
  double h0 = 0.0, h1 = 0.0, w0[NC] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (live) side_w0<3>(Ws, a.fc, m2 ? -1.0 : 1.0, gs, h0, h1, w0);
  double W0[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) W0[q] = w0[q] + lane_xor<1>(w0[q]);
  SidePart<3, double> P, T;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) P.dW0[d][q] = 0.0;
    P.S1[q] = P.S2[q] = P.S3[q] = 0.0;
  }
  P.H1 = P.H2 = P.H3 = 0.0;
  bool ok = true;
  double ps = 0.0;
  if (live) {
    make_gas<3>(W0, a.fc.N, g0);
    side_part<3, NS>(gs, h0, h1, Ws, dWs, a.fc, g0, P);
    ok = gs.ok && g0.ok;
    ps = gs.rho * gs.h;
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) T.dW0[d][q] = P.dW0[d][q] + lane_xor<1>(P.dW0[d][q]);
    T.S1[q] = P.S1[q] + lane_xor<1>(P.S1[q]);
    T.S2[q] = P.S2[q] + lane_xor<1>(P.S2[q]);
    T.S3[q] = P.S3[q] + lane_xor<1>(P.S3[q]);
  }
  if (NS) {
    T.H1 = P.H1 + lane_xor<1>(P.H1);
    T.H2 = P.H2 + lane_xor<1>(P.H2);
    T.H3 = P.H3 + lane_xor<1>(P.H3);
  } else {
    T.H1 = T.H2 = T.H3 = 0.0;
  }
  const double pp = lane_xor<1>(ps);
  ok = ok && (lane_xor<1>((int)ok) != 0);
  double A[NC] = {0, 0, 0, 0, 0}, B[NC] = {0, 0, 0, 0, 0};
  if (live) {
    double Fdt[NC], Fh[NC];
    flux_combine<3, NS>(W0, g0, T, m2 ? pp : ps, m2 ? ps : pp, a.fc, dt, Fdt, Fh);
    if (!ok && m2 == 0) atomicAdd(a.fail, 1ull);
    write_combined<NC>(STAGE, Fdt, Fh, 0.25, A, B);
  }
  // sum over the four Gauss points (m3, m1); both lanes of a pair hold the
  // same flux
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    A[q] += lane_xor<2>(A[q]);
    A[q] += other_quad(A[q]);  // quads hold their sums after the two steps above
    if (STAGE == 1) {
      B[q] += lane_xor<2>(B[q]);
      B[q] += other_quad(B[q]);
    }
  }
  wall_fluxes<NC>(g, AX, fa, A, B);
  if (live && (tid & 7) == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      a.FA[(long long)perm[q] * nf + fid] = A[q];
      if (STAGE == 1) a.FB[(long long)perm[q] * nf + fid] = B[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Updates.  Face arrays of direction d: [nc][faces_d] with the face index of
// cell (i,j,k)'s low face equal to the cell index in a grid whose axis d has
// n[d] + 1 entries.
// ---------------------------------------------------------------------------
struct UpdateArgs {
  Geom g;
  const double* W;    // stage 1: W^n; stage 2: P
  double* out1;       // stage 1: W*; stage 2: W^{n+1}
  double* out2;       // stage 1: P
  const double* FA[3];
  const double* FB[3];
  const double* dt;
  double gamma, mu;
  double* partial;    // stage 2 with CFL: one minimum per block, or null
};

// minimum over the block (blockDim.x a multiple of 64, at most 1024);
// valid in thread 0
__device__ __forceinline__ double block_min(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = fmin(v, red[i]);
  }
  return v;
}

// local CFL limit of one cell (Sec. 5 preamble); NaN for a non-physical state
template <int D>
__device__ __forceinline__ double cell_dt(const double* w, double gamma, double mu, double dxm) {
  const double rho = w[0];
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double u = w[d + 1] / rho;
    ke += u * u;
  }
  const double p = (gamma - 1.0) * (w[D + 1] - 0.5 * rho * ke);
  if (!(rho > 0.0) || !(p > 0.0)) return NAN;
  double v = dxm / (sqrt(ke) + sqrt(gamma * p / rho));
  if (mu > 0.0) v = fmin(v, dxm * dxm * rho / (4.0 * mu));
  return v;
}

// cell id of this thread; the block's CFL minimum goes to *partial
template <int D, int STAGE, bool CFL>
__device__ __forceinline__ void update_body(const UpdateArgs& u, long long id, double* partial) {
  constexpr int NC = D + 2;
  __shared__ double red[16];  // one entry per wave, up to 1024 threads
  const Geom& g = u.g;
  const bool live = id < g.ncell;
  const double dt = *u.dt;
  const bool adv = dt > 0.0;
  double w1[NC];
  if (live) {
    const int i = (int)(id % g.n[0]);
    const int j = D >= 2 ? (int)((id / g.n[0]) % g.n[1]) : 0;
    const int k = D >= 3 ? (int)(id / ((long long)g.n[0] * g.n[1])) : 0;
    long long lo[3], hi[3], nf[3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int e0 = g.n[0] + (d == 0), e1 = g.n[1] + (d == 1);
      nf[d] = (long long)e0 * e1 * (g.n[2] + (d == 2));
      lo[d] = ((long long)k * e1 + j) * e0 + i;
      hi[d] = lo[d] + (d == 0 ? 1 : d == 1 ? (long long)e0 : (long long)e0 * e1);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double w = u.W[(long long)c * g.ncell + id];
      double a = w, b = w;
      if (adv) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const double* FA = u.FA[d] + (long long)c * nf[d];
          a -= (FA[hi[d]] - FA[lo[d]]) / g.dx[d];
          if (STAGE == 1) {
            const double* FB = u.FB[d] + (long long)c * nf[d];
            b -= (FB[hi[d]] - FB[lo[d]]) / g.dx[d];
          }
        }
      }
      u.out1[(long long)c * g.ncell + id] = a;
      if (STAGE == 1) u.out2[(long long)c * g.ncell + id] = b;
      w1[c] = a;
    }
  }
  if (CFL) {
    double dxm = g.dx[0];
    for (int d = 1; d < D; ++d) dxm = fmin(dxm, g.dx[d]);
    double v = live ? cell_dt<D>(w1, u.gamma, u.mu, dxm) : INFINITY;
    // NaN (non-physical cell) wins the reduction
    const bool nan = live && !(v == v);
    v = block_min(nan ? -INFINITY : v, red);
    if (threadIdx.x == 0) *partial = v == -INFINITY ? NAN : v;
  }
}

template <int D, int STAGE, bool CFL>
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs u) {
  update_body<D, STAGE, CFL>(u, (long long)blockIdx.x * blockDim.x + threadIdx.x,
                            CFL ? u.partial + blockIdx.x : nullptr);
}

// CFL partial minima of a state (no update)
template <int D>
__device__ __forceinline__ void cfl_partial_body(const Geom& g, const double* W, double gamma, double mu,
                                                 long long id, double* partial) {
  constexpr int NC = D + 2;
  __shared__ double red[16];  // one entry per wave, up to 1024 threads
  double dxm = g.dx[0];
  for (int d = 1; d < D; ++d) dxm = fmin(dxm, g.dx[d]);
  double v = INFINITY;
  bool nan = false;
  if (id < g.ncell) {
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = W[(long long)c * g.ncell + id];
    v = cell_dt<D>(w, gamma, mu, dxm);
    nan = !(v == v);
  }
  v = block_min(nan ? -INFINITY : v, red);
  if (threadIdx.x == 0) *partial = v == -INFINITY ? NAN : v;
}

template <int D>
__global__ __launch_bounds__(256) void cfl_partial_kernel(Geom g, const double* W, double gamma, double mu,
                                                          double* partial) {
  cfl_partial_body<D>(g, W, gamma, mu, (long long)blockIdx.x * blockDim.x + threadIdx.x, partial + blockIdx.x);
}

// Final reduction.  clock = {t, dt}.  mode 0: dt_out = cfl * min (clipped to
// t_end - t_in); mode 1 (after a step): t += dt, then the next dt as mode 0;
// mode 2: fixed step, t += dt only.
__device__ __forceinline__ void finalize_body(const double* partial, int nblk, double cfl, double t_in,
                                              double t_end, double* clock, double* dt_out, int mode) {
  __shared__ double red[16];  // one entry per wave, up to 1024 threads
  double v = INFINITY;
  bool nan = false;
  if (mode != 2)
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
      const double p = partial[i];
      if (!(p == p)) nan = true;
      v = fmin(v, p);
    }
  v = block_min(nan ? -INFINITY : v, red);
  if (threadIdx.x == 0) {
    double t = t_in;
    if (mode >= 1) {
      t = clock[0];
      const double used = clock[1];
      if (used > 0.0) t += used;
    }
    if (clock) clock[0] = t;
    if (mode != 2) {
      double dt = v == -INFINITY ? NAN : cfl * v;
      if (t_end > 0.0) {
        if (t >= t_end * (1.0 - 1e-14))
          dt = 0.0;
        else if (t + dt > t_end)
          dt = t_end - t;
      }
      if (clock) clock[1] = dt;
      if (dt_out) *dt_out = dt;
    }
  }
}

static __global__ __launch_bounds__(256) void cfl_finalize_kernel(const double* partial, int nblk, double cfl,
                                                           double t_in, double t_end, double* clock,
                                                           double* dt_out, int mode) {
  finalize_body(partial, nblk, cfl, t_in, t_end, clock, dt_out, mode);
}

// clears n counters (a kernel rather than a memset, so that a caller may
// capture it into a graph)
static __global__ __launch_bounds__(256) void zero_counters_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

static __global__ void set_clock_kernel(double* clock, double t, double dt) {
  clock[0] = t;
  clock[1] = dt;
}

}  // namespace tgks
