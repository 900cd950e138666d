// Force kernels of the shifted-force variant of the Gaussian pair form (see ljmd_force.h).
#include "ljmd_force.h"

namespace ljmd {

hipError_t launch_force_gauss_sf(hipStream_t s, const ForceArgs &a, int prec, int tpp, int mode,
                               bool energy, int block) {
    return launch_force_style<STYLE_GAUSS | STYLE_SF>(s, a, prec, tpp, mode, energy, block);
}

}  // namespace ljmd
