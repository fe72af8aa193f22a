// The FP32 one-wavefront backward sweep of the 4-qubit 4-level layout without dipole terms
// (k_backward<float, 4, 4, 3, false>), compiled on its own so that it can take the instruction
// scheduler's ILP strategy (build.py passes it for this file only).  That kernel runs two
// wavefronts per SIMD, fixed by its 2048 items per launch, so registers beyond its current
// use cost no occupancy, and a schedule that spreads independent instructions further apart
// shortens its steps; for other kernels the same strategy raises register use past an
// occupancy step or into scratch.  Everything else is built from qoc_kernels.hip as usual,
// which takes this kernel's address from backward_q4l4_fp32().
#define QOC_BACKWARD_UNIT
#include "qoc_kernels.hip"
