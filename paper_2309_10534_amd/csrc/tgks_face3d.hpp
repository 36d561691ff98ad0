// tgks_face3d.hpp -- launches of the 3-D normal reconstruction and face
// kernels of one direction (instantiated once per direction in
// tgks_face3d_{x,y,z}.hip, so that the three compile in parallel).
#pragma once
#include "tgks_internal.hpp"

template <int AX>
int launch_face3d_ax(tgks_ctx* c, const StageArgs& a, int stage, bool fl) {
  int ext[3] = {c->g.n[0], c->g.n[1], c->g.n[2]};
  ext[AX] += 2;
  const long long nr = (long long)ext[0] * ext[1] * ext[2];
  {
    Timer tm(c, 3);
    dim3 grid((unsigned)((nr * 5 + 255) / 256));
    if (fl)
      hipLaunchKernelGGL((recon3d_kernel<AX, true>), grid, dim3(256), 0, c->stream, a);
    else
      hipLaunchKernelGGL((recon3d_kernel<AX, false>), grid, dim3(256), 0, c->stream, a);
  }
  {
    Timer tm(c, AX);
    const int n1 = c->g.n[(AX + 1) % 3], n2 = c->g.n[(AX + 2) % 3];
    const long long nbl = (long long)(c->g.n[AX] + 1) * ((n1 + B3_1 - 1) / B3_1) * ((n2 + B3_2 - 1) / B3_2);
    const dim3 grid((unsigned)(8 * ((nbl + 7) / 8))), blk3(L3 * B3_1 * B3_2);
#define F3L(...) hipLaunchKernelGGL((face3d_kernel<__VA_ARGS__>), grid, blk3, 0, c->stream, a)
#define F3(EXV)                                  \
  if (stage == 1 && fl) {                        \
    if (c->ns) F3L(AX, 1, true, EXV, true);      \
    else F3L(AX, 1, false, EXV, true);           \
  } else if (stage == 1) {                       \
    if (c->ns) F3L(AX, 1, true, EXV, false);     \
    else F3L(AX, 1, false, EXV, false);          \
  } else {                                       \
    if (c->ns) F3L(AX, 2, true, EXV, false);     \
    else F3L(AX, 2, false, EXV, false);          \
  }
    // c->ex: the first-order fallback (3-D grids have no prescribed sides)
    if (c->ex) {
      F3(true)
    } else {
      F3(false)
    }
#undef F3
#undef F3L
  }
  HIPCHK(hipGetLastError());
  return TGKS_OK;
}
