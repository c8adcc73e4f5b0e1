// FP32 instantiation of the grid pipeline (mixed-precision plans).
#include "pipeline.h"

namespace ibdl {
std::unique_ptr<PreparedPass> prepare_f32(const std::vector<PassJob>& jobs) { return prepare_t<float>(jobs); }
// complex elements per line of the tiled half spectrum: tiles x columns per tile
int tile_pitch_f32(int n) { return col_tiles<float>(n) * col_width<float>(n); }
int col_width_f32(int n) { return col_width<float>(n); }
int z_rows_f32(int n) { return z_rows<float>(n); }
}  // namespace ibdl
