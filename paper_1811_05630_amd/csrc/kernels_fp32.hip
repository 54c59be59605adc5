// The amplitude kernels again, as namespace cq::f32: every value of the
// working form and every result of the gate arithmetic rounded to FP32
// (SIM_FP32).
#define CQ_FP32 1
#include "kernels.hip"
