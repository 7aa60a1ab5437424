// Wilson-clover apply variants beyond launch_dirac.
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// out = D in for nrhs fields: in FP32, out and the arithmetic FP64 (the FP64
// links and clover term; each input value widened exactly). The same numbers
// as launch_convert to FP64 followed by launch_dirac in FP64.
int launch_dirac_widen(Ctx *c, int nrhs, const void *in32, void *out64);

}  // namespace mgdd
