// Stage kernels for order 3 (Venkatakrishnan), psi stored as bf16 (instantiations of sn_stage_impl.h).
#include "sn_stage_impl.h"

namespace snk {

hipError_t launch_stage_o3_bf16(int mode, int rows, int waves, const StageArgs& a, hipStream_t s) {
    return launch_stage_tu<3, uint16_t>(mode, rows, waves, a, s);
}

hipError_t launch_batch_o3_bf16(int mode, int rows, int waves, const BatchLaunch& L, int wgs_per_cu, int cus,
                               int face_lds, hipStream_t s) {
    return launch_batch_tu<3, uint16_t>(mode, rows, waves, L, wgs_per_cu, cus, face_lds, s);
}

}  // namespace snk
