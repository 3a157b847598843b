// Sweep kernels of EOS kind 1: the explicit instances of their launchers.
#include "shasta_sweeps.hpp"

namespace shasta {
SHASTA_SCHEMES_EOS1()
}  // namespace shasta
