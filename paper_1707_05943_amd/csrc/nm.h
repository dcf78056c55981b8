// Internal declarations of the non-Markovian measures' readouts (not installed).
#pragma once

#include "fdtd_common.h"

// N_geo of App. D over rows 0..R into dst (device); stages mu and lambda of
// rows 0..R in the context's Mu and Pe buffers on the way
int launch_ngeo(fdtd_ctx* c, int64_t R, double* dst);
