// adjoint.hip -- placeholder translation unit for the soft-kick adjoint.
#include "p3t_internal.h"
