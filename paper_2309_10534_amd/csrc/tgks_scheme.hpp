// tgks_scheme.hpp -- launches of the face kernels of the paper's comparison
// schemes (WENO-AO, TENO5, WENO-Z; 1-D and 2-D grids, conservative
// variables), instantiated once per scheme in tgks_scheme_{ao,teno5,wenoz}.hip.
#pragma once
#include "tgks_internal.hpp"

// a: the stage arguments of each direction (a[0] x faces, a[1] y faces)
template <int SCHEME>
int launch_scheme_faces(tgks_ctx* c, const StageArgs* a, int stage, bool fl) {
  if (c->g.D == 1) {
    Timer tm(c, 0);
    const dim3 grid((unsigned)((c->g.n[0] + 1 + 255) / 256)), blk(256);
#define L1(...) hipLaunchKernelGGL((face1d_kernel<__VA_ARGS__>), grid, blk, 0, c->stream, a[0])
    if (stage == 1 && fl) {
      if (c->ns) L1(1, true, true, false, false, SCHEME);
      else L1(1, false, true, false, false, SCHEME);
    } else if (stage == 1) {
      if (c->ns) L1(1, true, false, false, false, SCHEME);
      else L1(1, false, false, false, false, SCHEME);
    } else {
      if (c->ns) L1(2, true, false, false, false, SCHEME);
      else L1(2, false, false, false, false, SCHEME);
    }
#undef L1
  } else {
    Timer tm(c, 0);
    constexpr int TILE = CHAR_TILE2;
    constexpr int TN = tile2_tn(TILE), TT = tile2_tt(TILE);
    const int nx = c->g.n[0], ny = c->g.n[1];
    const long long nb = (long long)((nx + 1 + TN - 1) / TN) * ((ny + TT - 1) / TT) +
                         (long long)((ny + 1 + TN - 1) / TN) * ((nx + TT - 1) / TT);
    const dim3 grid((unsigned)nb), block(2 * TN * TT);
#define L2(...) hipLaunchKernelGGL((face2d_xy_kernel<__VA_ARGS__>), grid, block, 0, c->stream, a[0], a[1])
    if (stage == 1 && fl) {
      if (c->ns) L2(1, true, true, TILE, false, false, SCHEME);
      else L2(1, false, true, TILE, false, false, SCHEME);
    } else if (stage == 1) {
      if (c->ns) L2(1, true, false, TILE, false, false, SCHEME);
      else L2(1, false, false, TILE, false, false, SCHEME);
    } else {
      if (c->ns) L2(2, true, false, TILE, false, false, SCHEME);
      else L2(2, false, false, TILE, false, false, SCHEME);
    }
#undef L2
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}
