// Wavefront-cooperative engine for four stacked coordinated-turn targets
// (nx = 20) seen by eight bearing sensors, with sigma-point linearisation, FP64.
#include "dense_engine.hpp"

namespace pks {

EngineBase* make_engine_dense_ct_f64(int nx, int ny) {
  if (nx == 20 && ny == 8) return new DenseEngine<CtBearings<20, 8, double>, double>();
  return nullptr;
}

}  // namespace pks
