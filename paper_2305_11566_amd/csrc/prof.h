// Per-stage timing hook (see sv_profile_enable in sv.h).
#pragma once

#include "common.h"

namespace sv {

enum ProfStage {
    PROF_CENSUS = 0, PROF_COST_WTA, PROF_E1, PROF_E2, PROF_E3, PROF_HEAD, PROF_REPARAM, PROF_G3,
    PROF_G2, PROF_G1, PROF_G0, PROF_FPROJ, PROF_FINAL, PROF_SPLIT, PROF_NSTAGES
};

// Records the start (which = 0) or end (1) event of `stage` on `st` when
// profiling is enabled; a no-op otherwise.
void prof_mark(int stage, int which, hipStream_t st);

// How many times a profiled stage is launched back to back between its two
// events: the sv_profile_repeat setting while profiling is on, else 1.  Every
// stage rewrites the same outputs from the same inputs, so a repeat leaves
// the results unchanged.
int prof_repeat();

}  // namespace sv
