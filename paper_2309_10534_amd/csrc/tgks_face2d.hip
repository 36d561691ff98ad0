// tgks_face2d.hip -- launches of the 2-D face kernel (all directions,
// stages and tile shapes), compiled apart from the rest of the library.
#include "tgks_internal.hpp"

using namespace tgks;

#define LAUNCH(kern, grid, block, args) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, args)

// 2-D face kernel of one direction, stage and tile shape
template <int TILE>
static void launch_face2d(tgks_ctx* c, const StageArgs& a, int ax, int stage, bool fl, int nN, int nT) {
  constexpr int TN = tile2_tn(TILE), TT = tile2_tt(TILE);
  const dim3 grid((unsigned)((nN + 1 + TN - 1) / TN), (unsigned)((nT + TT - 1) / TT)), block(2 * TN * TT);
#define F2(AXV)                                                                                     \
  if (stage == 1) {                                                                                 \
    if (fl) {                                                                                       \
      if (c->ns) LAUNCH((face2d_kernel<AXV, 1, true, true, TILE>), grid, block, a);                 \
      else LAUNCH((face2d_kernel<AXV, 1, false, true, TILE>), grid, block, a);                      \
    } else {                                                                                        \
      if (c->ns) LAUNCH((face2d_kernel<AXV, 1, true, false, TILE>), grid, block, a);                \
      else LAUNCH((face2d_kernel<AXV, 1, false, false, TILE>), grid, block, a);                     \
    }                                                                                               \
  } else {                                                                                          \
    if (c->ns) LAUNCH((face2d_kernel<AXV, 2, true, false, TILE>), grid, block, a);                  \
    else LAUNCH((face2d_kernel<AXV, 2, false, false, TILE>), grid, block, a);                       \
  }
  if (ax == 0) {
    F2(0)
  } else {
    F2(1)
  }
#undef F2
}

// both directions of one stage in one launch
template <int TILE>
static void launch_face2d_xy(tgks_ctx* c, const StageArgs& ax, const StageArgs& ay, int stage, bool fl) {
  constexpr int TN = tile2_tn(TILE), TT = tile2_tt(TILE);
  const int nx = c->g.n[0], ny = c->g.n[1];
  const long long nb = (long long)((nx + 1 + TN - 1) / TN) * ((ny + TT - 1) / TT) +
                       (long long)((ny + 1 + TN - 1) / TN) * ((nx + TT - 1) / TT);
  const dim3 grid((unsigned)nb), block(2 * TN * TT);
#define LXY(kern) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, ax, ay)
  if (stage == 1) {
    if (fl) {
      if (c->ns) LXY((face2d_xy_kernel<1, true, true, TILE>));
      else LXY((face2d_xy_kernel<1, false, true, TILE>));
    } else {
      if (c->ns) LXY((face2d_xy_kernel<1, true, false, TILE>));
      else LXY((face2d_xy_kernel<1, false, false, TILE>));
    }
  } else {
    if (c->ns) LXY((face2d_xy_kernel<2, true, false, TILE>));
    else LXY((face2d_xy_kernel<2, false, false, TILE>));
  }
#undef LXY
}

// characteristic variables, prescribed sides or the fallback: one tile shape
template <bool CH, bool EX>
static void launch_face2d_xy_one(tgks_ctx* c, const StageArgs& ax, const StageArgs& ay, int stage, bool fl) {
  constexpr int TILE = CHAR_TILE2;
  constexpr int TN = tile2_tn(TILE), TT = tile2_tt(TILE);
  const int nx = c->g.n[0], ny = c->g.n[1];
  const long long nb = (long long)((nx + 1 + TN - 1) / TN) * ((ny + TT - 1) / TT) +
                       (long long)((ny + 1 + TN - 1) / TN) * ((nx + TT - 1) / TT);
  const dim3 grid((unsigned)nb), block(2 * TN * TT);
#define LXY(kern) hipLaunchKernelGGL(kern, grid, block, 0, c->stream, ax, ay)
  if (stage == 1) {
    if (fl) {
      if (c->ns) LXY((face2d_xy_kernel<1, true, true, TILE, CH, EX>));
      else LXY((face2d_xy_kernel<1, false, true, TILE, CH, EX>));
    } else {
      if (c->ns) LXY((face2d_xy_kernel<1, true, false, TILE, CH, EX>));
      else LXY((face2d_xy_kernel<1, false, false, TILE, CH, EX>));
    }
  } else {
    if (c->ns) LXY((face2d_xy_kernel<2, true, false, TILE, CH, EX>));
    else LXY((face2d_xy_kernel<2, false, false, TILE, CH, EX>));
  }
#undef LXY
}

int launch_face2d_xy_any(tgks_ctx* c, const StageArgs& ax, const StageArgs& ay, int stage, bool fl) {
  const bool ch = c->p.recon == TGKS_RECON_CHARACTERISTIC, ex = c->ex;
  if (ch || ex) {
    if (ch && ex) launch_face2d_xy_one<true, true>(c, ax, ay, stage, fl);
    else if (ch) launch_face2d_xy_one<true, false>(c, ax, ay, stage, fl);
    else launch_face2d_xy_one<false, true>(c, ax, ay, stage, fl);
    return TGKS_OK;
  }
  switch (c->tile2) {
    case 1:
      launch_face2d_xy<1>(c, ax, ay, stage, fl);
      break;
    case 2:
      launch_face2d_xy<2>(c, ax, ay, stage, fl);
      break;
    default:
      launch_face2d_xy<0>(c, ax, ay, stage, fl);
  }
  return TGKS_OK;
}

int launch_face2d_any(tgks_ctx* c, const StageArgs& a, int ax, int stage, bool fl) {
  if (c->ex || c->p.recon == TGKS_RECON_CHARACTERISTIC) return TGKS_EINVAL;  // merged launch only
  const int nN = c->g.n[ax], nT = c->g.n[1 - ax];
  switch (c->tile2) {
    case 1:
      launch_face2d<1>(c, a, ax, stage, fl, nN, nT);
      break;
    case 2:
      launch_face2d<2>(c, a, ax, stage, fl, nN, nT);
      break;
    default:
      launch_face2d<0>(c, a, ax, stage, fl, nN, nT);
  }
  return TGKS_OK;
}
