// Wilson-clover apply variants beyond launch_dirac.
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

// out = D in for nrhs fields: in FP32 (in_prec MGDD_F32) or half precision
// (MGDD_F16), out and the arithmetic FP64 (the FP64 links and clover term;
// each input value widened exactly). The same numbers as launch_convert to
// FP64 followed by launch_dirac in FP64.
int launch_dirac_widen(Ctx *c, int nrhs, const void *in, void *out64, int in_prec = MGDD_F32);

}  // namespace mgdd
