// tgks_scheme_ao.hip -- face kernels of the WENO-AO GKS (see tgks_scheme.hpp).
#include "tgks_scheme.hpp"

template int launch_scheme_faces<SCHEME_WENO_AO>(tgks_ctx* c, const StageArgs* a, int stage, bool fl);
