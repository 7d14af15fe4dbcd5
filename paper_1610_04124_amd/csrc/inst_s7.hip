// Recurrence kernels of 7 64-row slot(s) per lane (columns of up to 448 rows).
#define STX_SLOTS 7
#include "inst_body.h"
