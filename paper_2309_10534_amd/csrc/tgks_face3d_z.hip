// tgks_face3d_z.hip -- 3-D kernels of the z faces (see tgks_face3d.hpp).
#include "tgks_face3d.hpp"

template int launch_face3d_ax<2>(tgks_ctx* c, const StageArgs& a, int stage, bool fl);
