// FP64 instantiation of the grid pipeline.
#include "pipeline.h"

namespace ibdl {
std::unique_ptr<PreparedPass> prepare_f64(const std::vector<PassJob>& jobs) { return prepare_t<double>(jobs); }
// complex elements per line of the tiled half spectrum: tiles x columns per tile
int tile_pitch_f64(int n) { return col_tiles<double>(n) * col_width<double>(n); }
int col_width_f64(int n) { return col_width<double>(n); }
int z_rows_f64(int n) { return z_rows<double>(n); }
}  // namespace ibdl
