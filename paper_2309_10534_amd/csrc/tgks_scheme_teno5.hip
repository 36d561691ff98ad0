// tgks_scheme_teno5.hip -- face kernels of the TENO5 GKS (see tgks_scheme.hpp).
#include "tgks_scheme.hpp"

template int launch_scheme_faces<SCHEME_TENO5>(tgks_ctx* c, const StageArgs* a, int stage, bool fl);
