// ems_kernels_slab_f32.hip -- the mixed-form (FP32) kernels of the slab
// stack: the same templates as ems_kernels.hip, instantiated here for float
// and geometry kind 0 only, so that build.py can compile them with another
// instruction scheduler (one that favours independent instructions over
// register pressure).  On the 10^5-event beam that shortened the mixed
// e-/e+ launch by 4%; the FP64 kernels and the box-geometry kernels ran
// slower with it and keep the default.  The instruction order is all that
// changes: every arithmetic operation, and so every result, is the same.
#define EMS_SLAB_F32_TU 1
#include "ems_kernels.hip"
