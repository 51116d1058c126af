"""CPU oracle for the NGP-RT rendering hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, independent implementation of what the renderer computes,
written from the paper (arXiv 2407.10482): occupancy-distance marching
(Sec. 4.3, Eq. 9), trilinear hash-table lookups (Sec. 3 Eq. 3, Sec. 4.1
Eq. 6), attention across levels (Sec. 4.2, Eq. 7-8, in the softmax form used
here), front-to-back compositing (Sec. 3 Eq. 2 and Eq. 5), the deferred MLP
(Eq. 5, supplement "Network Design"), plus the reduced-precision tables,
the analytic gradients and the proposal network.

Values are computed in float64.  Where floating point decides an integer
(which lattice points are sampled, when transmittance crosses the
termination threshold) the decision is taken in a float32 mirror of the
renderer's arithmetic, op by op, so that integer outputs can be compared bit
for bit.

Only the tests, the smoke check and the benchmark's CPU baseline may import
this package.  It shares no code with the GPU library and never calls it.
"""
