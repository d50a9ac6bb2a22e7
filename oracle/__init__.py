"""FP64 CPU oracle for the qudit state-vector hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library (``paper_2409_17716_amd``) and imports nothing from it; the only
module both sides read is ``qf_inputs``, which holds gate descriptors and seeded
random draws but no gate arithmetic.

Everything here is plain NumPy in complex128 / float64 and follows the paper's
definitions directly (Appendix "Matrix form of the quantum gates"):

* ``gates``   - the gate matrices: generalized NOT, phase-shift (clock), Fourier,
                generalized Gell-Mann generators, rotations exp(-i theta S / 2)
                computed by eigendecomposition of the Hermitian generator.
* ``sim``     - basis states in the decimal representation, application of
                one-qudit / k-qudit matrices, digit permutations (CNOT = CSUM) and
                diagonal phases, and a gate-by-gate circuit runner.
* ``measure`` - probabilities, marginal probabilities and diagonal expectations.
* ``grad``    - adjoint-method gradient (gate by gate) and central finite
                differences.
* ``brute``   - full D^n x D^n circuit unitaries for tiny n, built from the
                paper's sparse digit rules and Kronecker products, as an
                independent second route.
* ``mixed``   - registers of per-qudit dimensions (mixed radix): gates,
                measurement and the adjoint gradient, with the readings of the
                two-qudit gates across dimensions stated in its header.

Parity status of each function is recorded in its docstring; every function
is pinned (``tests/test_oracle_pins.py``, ``tests/test_oracle_mixed.py``).
"""
from . import gates, sim, measure, grad, brute, mixed  # noqa: F401
