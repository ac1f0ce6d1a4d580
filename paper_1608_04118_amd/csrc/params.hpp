// Host-side parameter handling shared by the translation units of the
// library.  Not part of the public ABI.
#pragma once

#include "lbm_ltne.h"

namespace ltne {

// Records a detailed message for lbm_ltne_last_error() and returns code.
int set_error(int code, const char* fmt, ...);
const char* last_error();
void clear_error();

// Validates p and fills d; tmin / tmax bound every initial and wall
// temperature (they set the automatic shift reference).
int derive(const lbm_ltne_params* p, double tmin, double tmax, lbm_ltne_derived* d);

// Range of the uniform initial and Dirichlet wall temperatures.
void temperature_range(const lbm_ltne_params* p, double* tmin, double* tmax);

// Wall whose Nusselt number is reported, or -1.
int hot_wall(const lbm_ltne_params* p);

}  // namespace ltne
