"""FP64 CPU oracle for boundary-MPS contraction and sampling of a 2D PEPS.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library shares no code with
it and never calls it.

Plain, slow, obviously correct NumPy (complex128) following Rudolph & Tindall,
"Simulating and Sampling from Quantum Circuits with 2D Tensor Networks":

* ``statevector``  -- exact amplitudes by full contraction (the definition);
* ``boundary``     -- one-site-fit boundary MPS through the rows of the norm
                      network, the stored boundary set, and the norm
                      (Methods, boundary MPS; Appendix, sampling, Fig. 7c-d);
* ``sampler``      -- row-by-row sampling with conditioned amplitude
                      boundaries, q(x) and p(x) (Appendix, sampling);
* ``environments`` -- one-site density matrices, <Z>, nearest-neighbour <ZZ>
                      (Results, Fig. 4: direct contraction);
* ``verify``       -- independent p(x) by a separate single-layer contraction
                      of <x|psi>, the norm estimate E_q[p/q], the sample KLD
                      and importance-sampled <Z> (Methods, sampling; Eq. kld);
* ``philox``       -- Philox4x64-10 (Salmon et al. 2011) for random initial
                      guesses and draws;
* ``bp``           -- belief propagation on the norm network, the BP norm
                      estimate and the loop BP error (Methods, Eqs. avBPError
                      and loopBPerror; Appendix, message update);
* ``circuit``      -- two-qubit gates by BP-gauged simple update, the gate
                      error and the fidelity estimate (Methods, circuit
                      simulation, Eqs. error_per_gate and total_fidelity).

Pins (tests marked ``not gpu``): exact statevectors on lattices of <= 16
qubits, brute-force summation over bond assignments, NumPy's own Philox,
sum_x q(x) = 1 at truncated bond, gauge invariance, direction independence,
product-state and single-row closed forms, sample histograms within the
shot-noise bound. Outputs at truncated bond dimension are fixed only by the
algorithm's definition ("parity unpinned" beyond the invariants above).
"""
from .philox import philox4x64_10, philox4x64_10_vec, draw_uniform, draw_uniforms_vec  # noqa: F401
from .statevector import statevector, brute_force_amplitude  # noqa: F401
from .boundary import boundary_set, norm, fit_double, plan_bonds, flip_vertical  # noqa: F401
from .sampler import sample, sample_one, fit_single, SamplingError  # noqa: F401
from .environments import environments, z_expectation  # noqa: F401
from .verify import amplitude, amplitudes, sample_stats  # noqa: F401
from .bp import bp_messages, bp_log_norm, primitive_loops, loop_bp_error  # noqa: F401
from .circuit import simple_update, apply_gate, message_roots  # noqa: F401
