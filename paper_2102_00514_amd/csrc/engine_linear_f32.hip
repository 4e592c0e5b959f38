// Kernel instantiations for the LinearModel model in float.
#include "engine.hpp"

namespace pks {

EngineBase* make_engine_linear_f32(int nx, int ny) {
  if (nx == 1 && ny == 1) return new Engine<LinearModel<1, 1, float>, float>();
  if (nx == 3 && ny == 2) return new Engine<LinearModel<3, 2, float>, float>();
  if (nx == 5 && ny == 2) return new Engine<LinearModel<5, 2, float>, float>();
  return nullptr;
}

}  // namespace pks
