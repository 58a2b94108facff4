// Batched delay ensemble (persistent 1-D sweeps); see at_ens_* in atfd.h.
#include "atfd_internal.hpp"
