// FP32 instantiation of the grid pipeline (mixed-precision plans).
#include "pipeline.h"

namespace ibdl {
void run_pipeline_f32(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st) {
    run_pipeline_t<float>(p, nrhs, in, out, st);
}
}  // namespace ibdl
