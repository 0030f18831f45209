// The tracer's kernels with the cubic interpolation kernel (Sect. 3.2) in
// INTERP_NORMALIZE mode, instantiated in a translation unit of their own so that the
// build compiles the interpolation orders side by side.
#define QSQ_TRACE_HIGH_TU
#define QSQ_TRACE_HIGH_MODE 5
#include "trace.hip"
