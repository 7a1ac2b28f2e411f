// Learned eddy-viscosity closure kernels (placeholder translation unit).
#include "lbm_internal.h"
