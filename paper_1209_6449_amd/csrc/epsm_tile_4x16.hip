// Scan and expand kernels of the 4 x 16 KiB tile (see epsm_scan.h).
#include "epsm_scan.h"

EPSM_TILE_TU(4, 16)
