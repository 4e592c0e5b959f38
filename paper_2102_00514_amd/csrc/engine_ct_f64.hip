// Kernel instantiations for the CtBearings model in double.
#include "engine.hpp"

namespace pks {

EngineBase* make_engine_ct_f64(int nx, int ny) {
  if (nx == 5 && ny == 2) return new Engine<CtBearings<5, 2, double>, double>();
  return nullptr;
}

}  // namespace pks
