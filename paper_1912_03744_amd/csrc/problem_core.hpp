// problem_core.hpp -- what other translation units of the library may see of
// a single-instance problem (adi_problem): its device, stream, parameters,
// geometry arrays and field, plus one slot for an extension state (the
// nonlinear path keeps its buffers there).  Implemented in solver.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adi.h"
#include "device.hpp"

namespace adi {

struct ProblemCore {
  int device;
  hipStream_t stream;
  Params P;     // geometry, films, grid size (materials unused by extensions)
  Geom g;       // device geometry arrays (built on first use)
  double* T;    // the field, nz*nr, r fastest, 0 outside the domain
  double time;  // model time of the field
};

// Make the problem's device current, build its geometry if needed and fill
// *out.  Fails like the other entry points (ADI_EINVAL for a null handle).
adi_status problem_core(adi_problem p, ProblemCore* out);

// The field was advanced by an extension to model time `time` over `steps`
// steps: carried right-hand sides of the linear path are stale, the step
// counter and the time move on.
void problem_field_advanced(adi_problem p, double time, int64_t steps);

// Extension state: one pointer per problem, released with `destroy` by
// adi_destroy (and before the slot is replaced).
void* problem_ext(adi_problem p);
void problem_set_ext(adi_problem p, void* ext, void (*destroy)(void*));

}  // namespace adi
