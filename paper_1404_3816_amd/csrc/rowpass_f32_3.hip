// Row-pass instantiations: C_Q in float, p / 16 = 3 mod 4.
#define HIKF_RP_TQ float
#define HIKF_RP_SEL 3
#include "rowpass.h"
