// Stage kernels for order 1, psi stored as f32 (instantiations of sn_stage_impl.h).
#include "sn_stage_impl.h"

namespace snk {

hipError_t launch_stage_o1_f32(int mode, int rows, int waves, const StageArgs& a, hipStream_t s) {
    return launch_stage_tu<1, float>(mode, rows, waves, a, s);
}

hipError_t launch_batch_o1_f32(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s) {
    return launch_batch_tu<1, float>(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
}

}  // namespace snk
