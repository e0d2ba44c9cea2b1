// Valence eigenpairs of H on the device (setup of systems without given psi_v).
#include "engine.hpp"

namespace sth {

void Context::valence(const sth_system_desc&, int, double, int, double*, double*, int, double*,
                      int*) {
  set_error("sth_valence: not available in this build");
  throw Error(STH_E_INTERNAL);
}

}  // namespace sth
