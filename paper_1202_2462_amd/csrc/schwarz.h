// Schwarz variants of Section 2: red-black multiplicative (Algorithm 2.1) or
// additive, with MR(k) or GMRES(k) block solves (schwarz.hip).
#pragma once

#include "mgdd_internal.h"

namespace mgdd {

constexpr int SCHWARZ_GMRES_MAX = 3;   // GMRES steps per block solve (more spill registers)

struct SchwarzOpts {
    int nsweeps = 1;
    int k = 4;            // MR or GMRES steps per block solve
    int gmres = 0;        // block solver: 0 MR, 1 GMRES
    int additive = 0;     // 0 red-black multiplicative, 1 additive
};

// bytes of workspace launch_schwarz needs for nrhs fields of precision prec
size_t schwarz_work_bytes(const Ctx *c, int prec, int nrhs, const SchwarzOpts &o);
// o.nsweeps sweeps on (D - shift) z = b (z in/out); work: schwarz_work_bytes
// (additive only; may be null otherwise). Additive sweeps need shift = 0.
int launch_schwarz(Ctx *c, int prec, int nrhs, const SchwarzOpts &o, double sre, double sim, const void *b, void *z,
                   void *work);

}  // namespace mgdd
