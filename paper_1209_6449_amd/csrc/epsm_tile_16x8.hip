// Scan and expand kernels of the 16 x 8 KiB tile (see epsm_scan.h).
#include "epsm_scan.h"

EPSM_TILE_TU(16, 8)
