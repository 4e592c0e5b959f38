// Wavefront-cooperative engine for four stacked coordinated-turn targets
// (nx = 20) seen by eight bearing sensors, with sigma-point linearisation, FP32.
#include "dense_engine.hpp"

namespace pks {

EngineBase* make_engine_dense_ct_f32(int nx, int ny) {
  if (nx == 20 && ny == 8) return new DenseEngine<CtBearings<20, 8, float>, float>();
  return nullptr;
}

}  // namespace pks
