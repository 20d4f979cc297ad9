// Stage kernels for order 2, psi stored as bf16 (instantiations of sn_stage_impl.h).
#include "sn_stage_impl.h"

namespace snk {

hipError_t launch_stage_o2_bf16(int mode, int rows, int waves, const StageArgs& a, hipStream_t s) {
    return launch_stage_tu<2, uint16_t>(mode, rows, waves, a, s);
}

hipError_t launch_batch_o2_bf16(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s) {
    return launch_batch_tu<2, uint16_t>(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
}

}  // namespace snk
