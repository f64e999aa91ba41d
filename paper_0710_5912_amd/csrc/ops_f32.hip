// Stage-kernel instantiations in FP32 (per-mode solves and reductions stay FP64).
#include "ops_impl.hpp"

namespace le {

bool get_ops_f32(int nx, int ny, Ops* ops) { return fill_ops<float>(nx, ny, ops); }

}  // namespace le
