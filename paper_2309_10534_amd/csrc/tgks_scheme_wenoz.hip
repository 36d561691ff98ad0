// tgks_scheme_wenoz.hip -- face kernels of the WENO-Z GKS (see tgks_scheme.hpp).
#include "tgks_scheme.hpp"

template int launch_scheme_faces<SCHEME_WENO_Z>(tgks_ctx* c, const StageArgs* a, int stage, bool fl);
