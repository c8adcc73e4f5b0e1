// FP32 instantiation of the grid pipeline (mixed-precision plans).
#include "pipeline.h"

namespace ibdl {
void run_pipeline_f32(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st) {
    run_pipeline_t<float>(p, nrhs, in, out, st);
}
// complex elements per line of the tiled half spectrum: tiles x columns per tile
int tile_pitch_f32(int n) { return col_tiles<float>(n) * col_width<float>(n); }
}  // namespace ibdl
