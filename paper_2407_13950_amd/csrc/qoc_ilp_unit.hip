// Kernel instances compiled on their own so that they can take the instruction scheduler's ILP
// strategy (build.py passes it for this file only); ilp_held() in qoc_kernels.hip lists them:
// the FP32 one-wavefront backward sweep of the 4-qubit 4-level layout, its forward sweep with
// dipole terms, and the sweeps that the default schedules run for the 2-qubit 3-level system in
// FP64 and the 3-qubit 4-level system in FP32.  The 4-qubit sweeps run two wavefronts per SIMD,
// fixed by their 2048 items per launch, and the others are latency-bound chains of a few
// wavefronts, so registers beyond their default use cost them no occupancy they need, and a
// schedule that spreads independent instructions further apart shortens their steps; for other
// kernels the same strategy lowers occupancy that their launches need, or spills.
// qoc_kernels.hip builds everything else and takes these kernels' addresses from ilp_kernels().
#define QOC_ILP_UNIT
#include "qoc_kernels.hip"
