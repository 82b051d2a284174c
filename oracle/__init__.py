"""FP64 CPU oracle for the finite-difference Landau-Lifshitz hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
double-precision restatement of what the solver computes.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  The GPU library never calls it and shares no code with it: the only
thing both sides consume is the seeded input generator module
(``workloads``), which holds no arithmetic of the method.

Everything here works in SI units (A/m, s, T, J), whereas the GPU library
works internally in reduced units; the two formulations meet only at the
C-ABI, which takes and returns SI quantities.

Modules and the passages of the paper (Vansteenkiste & Van de Wiele, MuMax)
that they follow:

* ``constants`` -- mu0, gamma, k_B (Sec. 2, Eq. 1 and Eq. 6).
* ``demag``     -- cell-averaged demagnetising tensor (Sec. 2.1.1, Eq. 2;
                   the tensor formula itself is not printed in the paper: the
                   Newell-Williams-Dunlop expressions are used near the source
                   cell and a tent-weighted quadrature of the point-dipole
                   tensor far from it), periodic images (Sec. 2.1.1), the
                   zero-padded FFT convolution and the direct O(N^2) sum.
* ``fields``    -- exchange (Sec. 2.1.2, Eq. 3), uniaxial and cubic
                   anisotropy (Sec. 2.1.3, Eq. 4-5), Zeeman, thermal field
                   (Sec. 2.1.3, Eq. 6), total H_eff and the energy.
* ``philox``    -- Philox4x32-10 counter-based generator (Salmon et al.,
                   SC'11) and the Box-Muller transform, for Eq. 6's eta.
* ``llg``       -- Landau-Lifshitz right-hand side (Sec. 2, Eq. 1) and the
                   Runge-Kutta integrators listed in Sec. 2.2 (Euler, Heun,
                   classical RK4, Dormand-Prince 5(4) with step control).

Parity unpinned (pinned only by self-consistency): which Philox counter a
cell and step draw from (a convention; the generator itself is pinned by
its known-answer vectors, the draws by their moments), and anything the
learned surrogate proposes.  The adaptive controller's step sequence is
pinned against scipy's independent Dormand-Prince and Bogacki-Shampine
solvers.
"""
