// Storage types of the CG vectors of an inner precision, shared by the
// solver's vector kernels and the hop that carries the fused CG step.
#pragma once

#include "common.h"

namespace qdwf {

// The inner residual r: FP16 for FP16 storage (r is kept at unit RMS like
// the other inner vectors, and its drift from b - A x between two reliable
// updates stays far below the update threshold), otherwise the compute
// type: FP32 for FP32 and BF16 storage (BF16 keeps too few bits for r),
// FP64 for FP64.
template <class S> struct ResidStore { typedef typename Store<S>::compute t; };
template <> struct ResidStore<_Float16> { typedef _Float16 t; };

}  // namespace qdwf
