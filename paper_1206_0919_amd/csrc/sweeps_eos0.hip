// Sweep kernels of EOS kind 0: the explicit instances of their launchers.
#include "shasta_sweeps.hpp"

namespace shasta {
SHASTA_SCHEMES_EOS0()
}  // namespace shasta
