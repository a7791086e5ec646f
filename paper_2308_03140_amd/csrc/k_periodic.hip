// placeholder translation unit (periodic kernels follow)
#include "mbd_internal.h"
