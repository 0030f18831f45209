// The tracer's general-geometry kernels (Sect. 3.1-3.2: spherical coordinates
// and rectilinear axes, stepped in physical coordinates) in INTERP_NORMALIZE mode,
// instantiated in a translation unit of their own.
#define QSQ_TRACE_HIGH_TU
#define QSQ_TRACE_HIGH_MODE 9
#include "trace.hip"
