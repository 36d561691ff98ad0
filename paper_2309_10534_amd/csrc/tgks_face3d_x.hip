// tgks_face3d_x.hip -- 3-D kernels of the x faces (see tgks_face3d.hpp).
#include "tgks_face3d.hpp"

template int launch_face3d_ax<0>(tgks_ctx* c, const StageArgs& a, int stage, bool fl);
