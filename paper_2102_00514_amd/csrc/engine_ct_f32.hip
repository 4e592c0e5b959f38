// Kernel instantiations for the CtBearings model in float.
#include "engine.hpp"

namespace pks {

EngineBase* make_engine_ct_f32(int nx, int ny) {
  if (nx == 5 && ny == 2) return new Engine<CtBearings<5, 2, float>, float>();
  return nullptr;
}

}  // namespace pks
