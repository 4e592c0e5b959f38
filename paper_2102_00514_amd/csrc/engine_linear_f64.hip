// Kernel instantiations for the LinearModel model in double.
#include "engine.hpp"

namespace pks {

EngineBase* make_engine_linear_f64(int nx, int ny) {
  if (nx == 1 && ny == 1) return new Engine<LinearModel<1, 1, double>, double>();
  if (nx == 3 && ny == 2) return new Engine<LinearModel<3, 2, double>, double>();
  if (nx == 5 && ny == 2) return new Engine<LinearModel<5, 2, double>, double>();
  return nullptr;
}

}  // namespace pks
