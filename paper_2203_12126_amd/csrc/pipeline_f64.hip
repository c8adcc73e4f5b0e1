// FP64 instantiation of the grid pipeline.
#include "pipeline.h"

namespace ibdl {
void run_pipeline_f64(ibdl_plan p, int nrhs, const PipeIn& in, const PipeOut& out, hipStream_t st) {
    run_pipeline_t<double>(p, nrhs, in, out, st);
}
// complex elements per line of the tiled half spectrum: tiles x columns per tile
int tile_pitch_f64(int n) { return col_tiles<double>(n) * col_width<double>(n); }
}  // namespace ibdl
