// tgks_batch.hpp -- batched S2O4 steps of many independent grids (1-D or 2-D)
// in one launch per kernel kind.
//
// The instances' states are packed one after another (each [nc][ny][nx]), and
// so are their face arrays.  Every launch walks a work list of (instance,
// local block) pairs built on the host; a block reads its instance's
// geometry and flux constants from a device table and runs the same tile,
// face or cell code as the single-grid kernels, so that a batched step is
// bit-identical to the same step of each grid alone.  Every instance has its
// own clock {t, dt} (its own CFL step) and failure counter.
#pragma once
#include "tgks_kernels.hpp"

namespace tgks {

struct BatchInst {
  Geom g;
  FluxCfg fc;
  TenoCfg tn, tt;
  double gamma, mu;
  long long woff;     // first double of the instance's state in a packed state
  long long foff[2];  // first double of its face arrays, per direction
  int ntile[2];       // 2-D: face tiles along the normal axis, per direction
  int blk0, nblk;     // its cell blocks (256 cells each) in the cell work list
};

struct BatchArgs {
  const BatchInst* inst;
  const int2* work;  // (instance, local block)
  const double* W;
  double* out1;
  double* out2;
  double* FA[2];
  double* FB[2];
  double* clock;     // [instance][t, dt]
  double* partial;   // per cell block
  unsigned long long* fail;  // per instance
  // first-order fallback, the same for every instance; a run-time value so
  // that the batched face code compiles as the single-grid code does
  int fallback;
};

__device__ __forceinline__ StageArgs batch_stage(const BatchArgs& b, const BatchInst& I, int inst, int ax) {
  StageArgs a;
  a.g = I.g;
  a.fc = I.fc;
  a.tn = I.tn;
  a.tt = I.tt;
  a.W = b.W + I.woff;
  a.FA = b.FA[ax] + I.foff[ax];
  a.FB = b.FB[ax] + I.foff[ax];
  a.dt = b.clock + 2 * inst + 1;
  a.fail = b.fail + inst;
  a.nflags = nullptr;
  a.tflags = nullptr;
  a.R = nullptr;
  a.Rout = nullptr;
  a.gamma = I.gamma;
  a.pb.on = 0;  // batches have no prescribed sides
  a.fallback = b.fallback;
  a.fbc = nullptr;  // fallbacks are not counted in batches
  a.t0 = 0.0;
  a.tclk = nullptr;
  return a;
}

template <int STAGE, bool NS, bool CHAR = false, bool EX = false>
__global__ __launch_bounds__(256) void batch_face1d_kernel(BatchArgs b) {
  const int2 w = b.work[blockIdx.x];
  const StageArgs a = batch_stage(b, b.inst[w.x], w.x, 0);
  face1d_body<STAGE, NS, false, CHAR, EX>(a, w.y * 256 + (int)threadIdx.x);
}

template <int AX, int STAGE, bool NS, int TILE, bool CHAR = false, bool EX = false>
__global__ __launch_bounds__(2 * tile2_tn(TILE) * tile2_tt(TILE), 2) void batch_face2d_kernel(BatchArgs b) {
  const int2 w = b.work[blockIdx.x];
  const BatchInst& I = b.inst[w.x];
  const StageArgs a = batch_stage(b, I, w.x, AX);
  const int nt = I.ntile[AX];
  __shared__ double lds[CHAR ? tile2_lds_char(TILE) : tile2_lds(TILE)];
  face2d_tile<AX, STAGE, NS, false, TILE, CHAR, EX>(a, w.y % nt, w.y / nt, lds);
}

template <int D, int STAGE, bool CFL>
__global__ __launch_bounds__(256) void batch_update_kernel(BatchArgs b) {
  const int2 w = b.work[blockIdx.x];
  const BatchInst& I = b.inst[w.x];
  UpdateArgs u;
  u.g = I.g;
  u.W = b.W + I.woff;
  u.out1 = b.out1 + I.woff;
  u.out2 = STAGE == 1 ? b.out2 + I.woff : nullptr;
  for (int d = 0; d < 3; ++d) {
    u.FA[d] = d < D ? b.FA[d] + I.foff[d] : nullptr;
    u.FB[d] = d < D ? b.FB[d] + I.foff[d] : nullptr;
  }
  u.dt = b.clock + 2 * w.x + 1;
  u.gamma = I.gamma;
  u.mu = I.mu;
  u.partial = nullptr;
  update_body<D, STAGE, CFL>(u, (long long)w.y * 256 + threadIdx.x, CFL ? b.partial + I.blk0 + w.y : nullptr);
}

template <int D>
__global__ __launch_bounds__(256) void batch_cfl_partial_kernel(BatchArgs b) {
  const int2 w = b.work[blockIdx.x];
  const BatchInst& I = b.inst[w.x];
  cfl_partial_body<D>(I.g, b.W + I.woff, I.gamma, I.mu, (long long)w.y * 256 + threadIdx.x,
                      b.partial + I.blk0 + w.y);
}

// one block per instance; mode as cfl_finalize_kernel (0: start at t = 0,
// 1: advance the clock and compute the next step).  steps[i] counts the steps
// instance i has taken (dt > 0) since the start.
static __global__ __launch_bounds__(256) void batch_finalize_kernel(const BatchInst* inst, const double* partial,
                                                                    double cfl, double t_end, double* clock,
                                                                    long long* steps, int mode) {
  const BatchInst& I = inst[blockIdx.x];
  double* ck = clock + 2 * blockIdx.x;
  if (threadIdx.x == 0) {
    if (mode == 0)
      steps[blockIdx.x] = 0;
    else if (ck[1] > 0.0)
      steps[blockIdx.x] += 1;
  }
  finalize_body(partial + I.blk0, I.nblk, cfl, 0.0, t_end, ck, nullptr, mode);
}

}  // namespace tgks
