// kernels_fast.hip — the fast-math build of the event kernels (Sec. 4.2: the
// paper's compiler fast-math switch).  Compiled with approximate
// transcendentals (v_log_f32, v_exp_f32, v_sqrt_f32), reciprocal division and
// flushed FP32 denormals; the tables the kernels read are the same as in the
// default build (setup.hip).
#define INC_KERNEL_NS fast
#include "kernels.hip"
