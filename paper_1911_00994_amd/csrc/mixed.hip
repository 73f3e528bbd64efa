// placeholder translation unit for the mixed-precision solver (filled in below)
#include "internal.h"
