// Discrete adjoint of the AT step; see at_adjoint* in atfd.h.
#include "atfd_internal.hpp"
