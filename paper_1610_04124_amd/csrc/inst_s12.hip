// Recurrence kernels of 12 64-row slot(s) per lane (columns of up to 768 rows).
#define STX_SLOTS 12
#include "inst_body.h"
