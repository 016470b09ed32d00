"""Plain FP64 CPU oracle for the D3Q27 chemical-potential free-energy
lattice Boltzmann step (Saito, Baba & Takada, arXiv:2504.03819).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this package: only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.  It
shares no code with the HIP library (no kernels, headers, tables or helpers).

Modules
-------
lattice      D3Q27 velocities and the weights of Eq. (17)
eos          van der Waals closure, Eqs. (29)-(32); Maxwell coexistence
lbm          the time step, Sec. II B, Eqs. (11)-(12), (18)-(28), the
             wetting boundary of Eqs. (36)-(38), and the initialiser
phase_space  the phase-space generalized equilibrium, Eqs. (13)-(16)
phys         measurement helpers: surface tension Eq. (33), discrete static
             equilibria by Newton, Young-Laplace prediction, radii, angles

Everything is float64 and written for readability, not speed.  The step is
written with plain torch CPU ops so that torch autograd can differentiate it:
the same code is the forward oracle and, through autograd, the reverse-mode
reference for the hand-written adjoint.
"""
