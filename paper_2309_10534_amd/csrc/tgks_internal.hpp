// tgks_internal.hpp -- host-side internals shared by the library's
// translation units: the context structure, error checking, parameter
// validation, per-launch timing and the launch helpers of the face kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "tgks.h"
#include "tgks_kernels.hpp"

using namespace tgks;

constexpr int NKIND = 7;

struct EventPair {
  hipEvent_t a, b;
};

struct tgks_ctx {
  tgks_params p;
  Geom g;
  FluxCfg fc;
  TenoCfg tn, tt;
  SchemeCfg sc;  // comparison schemes (p.scheme != TGKS_SCHEME_TENO_D)
  bool ns;
  int tile2 = 0;  // 2-D face-kernel tile shape (tile2_tn/tile2_tt index)
  hipStream_t stream;
  int nc;
  long long ncell;
  long long nface[3];
  double* Ws = nullptr;
  double* P = nullptr;
  double* W2 = nullptr;
  double* FA[3] = {nullptr, nullptr, nullptr};
  double* FB[3] = {nullptr, nullptr, nullptr};
  double* R = nullptr;
  double* partial = nullptr;
  int nblk = 0;
  double* clock = nullptr;
  unsigned long long* fail = nullptr;
  // prescribed sides: states, lines, and the time of the state being stepped
  // (t0 + *tclk; tclk is the run clock inside tgks_run, null otherwise)
  Prescribed pb{};
  double t0 = 0.0;
  const double* tclk = nullptr;
  bool ex = false;  // prescribed sides or the first-order fallback: the EX face kernels
  // graph cache of tgks_run
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int g_steps = -1;
  double g_cfl = 0, g_tend = 0, g_fixed = 0, g_t0 = 0;
  double* g_W = nullptr;
  double* g_time = nullptr;
  // reverse-mode buffers (allocated by the first tgks_step_adjoint)
  double* aGB = nullptr;
  uint8_t* aTF = nullptr;
  double* aNRB = nullptr;
  uint8_t* aNF = nullptr;
  double* aWsb = nullptr;
  // timing
  bool timing = false;
  std::vector<EventPair> ev[NKIND];
  std::vector<hipEvent_t> pool;
};

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      fprintf(stderr, "tgks: %s failed: %s\n", #x, hipGetErrorString(e_));         \
      return TGKS_EHIP;                                                            \
    }                                                                              \
  } while (0)

inline int check_params(const tgks_params* p) {
  if (!p || p->ndim < 1 || p->ndim > 3) return TGKS_EINVAL;
  for (int d = 0; d < 3; ++d) {
    if (d < p->ndim) {
      if (p->n[d] < 3 || !(p->dx[d] > 0.0)) return TGKS_EINVAL;
      if (p->bc_lo[d] < 0 || p->bc_lo[d] > 4 || p->bc_hi[d] < 0 || p->bc_hi[d] > 4) return TGKS_EINVAL;
      if ((p->bc_lo[d] == TGKS_BC_PERIODIC) != (p->bc_hi[d] == TGKS_BC_PERIODIC)) return TGKS_EINVAL;
      for (int e = 0; e < 2; ++e) {
        if ((e == 0 ? p->bc_lo[d] : p->bc_hi[d]) != TGKS_BC_PRESCRIBED) continue;
        if (p->ndim > 2) return TGKS_EINVAL;
        const int far = p->bc_far[d][e];
        if (far != TGKS_BC_TRANSMISSIVE && far != TGKS_BC_REFLECTIVE && far != TGKS_BC_PRESCRIBED)
          return TGKS_EINVAL;
        for (int k = 0; k < 3; ++k)
          if (std::isnan(p->bc_line[d][e][k])) return TGKS_EINVAL;
      }
    } else if (p->n[d] != 1) {
      return TGKS_EINVAL;
    }
  }
  if (!(p->gamma > 1.0) || !(p->mu >= 0.0) || !(p->prandtl > 0.0)) return TGKS_EINVAL;
  if (p->tau_mode < 0 || p->tau_mode > 2) return TGKS_EINVAL;
  if (p->tau_mode == TGKS_TAU_VISCOUS && !(p->mu > 0.0)) return TGKS_EINVAL;
  if (p->q < 1 || p->q > 16 || !(p->eps >= 0.0)) return TGKS_EINVAL;
  if (p->recon != TGKS_RECON_CONSERVATIVE && p->recon != TGKS_RECON_CHARACTERISTIC) return TGKS_EINVAL;
  if (p->recon == TGKS_RECON_CHARACTERISTIC && p->ndim > 2) return TGKS_EINVAL;
  if (p->fallback != 0 && p->fallback != 1) return TGKS_EINVAL;
  if (p->scheme < TGKS_SCHEME_TENO_D || p->scheme > TGKS_SCHEME_WENO_Z) return TGKS_EINVAL;
  if (p->scheme != TGKS_SCHEME_TENO_D) {
    // the comparison schemes: conservative variables on 1-D and 2-D grids,
    // no prescribed sides or fallback
    if (p->ndim > 2 || p->recon != TGKS_RECON_CONSERVATIVE || p->fallback != 0) return TGKS_EINVAL;
    for (int d = 0; d < p->ndim; ++d)
      if (p->bc_lo[d] == TGKS_BC_PRESCRIBED || p->bc_hi[d] == TGKS_BC_PRESCRIBED) return TGKS_EINVAL;
    if (p->scheme == TGKS_SCHEME_WENO_AO && !(p->d_hi > 0.0 && p->d_hi < 1.0 && p->d_lo > 0.0 && p->d_lo < 1.0))
      return TGKS_EINVAL;
    if (p->scheme != TGKS_SCHEME_TENO5 && !(p->eps_w > 0.0)) return TGKS_EINVAL;
  }
  double cells = 1.0;
  for (int d = 0; d < p->ndim; ++d) cells *= p->n[d];
  if (cells > 4.0e9) return TGKS_EINVAL;
  return TGKS_OK;
}

inline bool has_prescribed(const tgks_params* p) {
  for (int d = 0; d < p->ndim; ++d)
    if (p->bc_lo[d] == TGKS_BC_PRESCRIBED || p->bc_hi[d] == TGKS_BC_PRESCRIBED) return true;
  return false;
}

// kernel form of the prescribed sides (1-D and 2-D)
inline Prescribed prescribed_of(const tgks_params* p) {
  Prescribed b{};
  b.on = has_prescribed(p) ? 1 : 0;
  for (int d = 0; d < 2; ++d)
    for (int e = 0; e < 2; ++e) {
      b.far[d][e] = p->bc_far[d][e];
      for (int k = 0; k < 3; ++k) b.line[d][e][k] = p->bc_line[d][e][k];
    }
  for (int c = 0; c < 4; ++c) {
    b.A[c] = p->bc_state[0][c];
    b.B[c] = p->bc_state[1][c];
  }
  return b;
}

inline hipEvent_t take_event(tgks_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// begin/end markers around one launch of a kernel kind
struct Timer {
  tgks_ctx* c;
  int kind;
  hipEvent_t a = nullptr;
  Timer(tgks_ctx* c_, int k) : c(c_), kind(k) {
    if (c->timing) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~Timer() {
    if (c->timing && a) {
      hipEvent_t b = take_event(c);
      if (b) {
        (void)hipEventRecord(b, c->stream);
        c->ev[kind].push_back({a, b});
      }
    }
  }
};

inline StageArgs stage_args(tgks_ctx* c, const double* W, int ax, const double* dt) {
  StageArgs a;
  a.g = c->g;
  a.fc = c->fc;
  a.tn = c->tn;
  a.tt = c->tt;
  a.sc = c->sc;
  a.W = W;
  a.FA = c->FA[ax];
  a.FB = c->FB[ax];
  a.dt = dt;
  a.fail = c->fail;
  a.nflags = nullptr;
  a.tflags = nullptr;
  a.R = c->R;
  a.Rout = c->R;
  a.gamma = c->p.gamma;
  a.pb = c->pb;
  a.t0 = c->t0;
  a.tclk = c->tclk;
  a.fallback = c->p.fallback;
  a.fbc = c->fail + 1;  // the context's second counter
  return a;
}

// 2-D face kernels of one direction and stage (tgks_face2d.hip)
int launch_face2d_any(tgks_ctx* c, const StageArgs& a, int ax, int stage, bool fl);
int launch_face2d_xy_any(tgks_ctx* c, const StageArgs& ax, const StageArgs& ay, int stage, bool fl);

// face kernels of a comparison scheme, all directions of one stage
// (tgks_scheme_*.hip)
template <int SCHEME>
int launch_scheme_faces(tgks_ctx* c, const StageArgs* a, int stage, bool fl);

// 3-D normal reconstruction and face kernels of direction AX (tgks_face3d_*.hip)
template <int AX>
int launch_face3d_ax(tgks_ctx* c, const StageArgs& a, int stage, bool fl);

// host-side description of a grid without device memory (tgks_capi.hip)
void init_ctx_host(tgks_ctx* c, const tgks_params* p, void* stream);

// forward pieces of one step (tgks_capi.hip)
int do_step(tgks_ctx* c, const double* W, double* out, const double* dt, uint8_t* flags, bool cfl);
int launch_faces(tgks_ctx* c, const double* W, const double* dt, int stage, uint8_t* flags);
int launch_update(tgks_ctx* c, int stage, const double* W, double* o1, double* o2, const double* dt, bool cfl);
