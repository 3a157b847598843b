// Sweep kernels of EOS kind 2: the explicit instances of their launchers.
#include "shasta_sweeps.hpp"

namespace shasta {
SHASTA_SCHEMES_EOS2()
}  // namespace shasta
