// Sweep kernels of EOS kind 3: the explicit instances of their launchers.
#include "shasta_sweeps.hpp"

namespace shasta {
SHASTA_SCHEMES_EOS3()
}  // namespace shasta
