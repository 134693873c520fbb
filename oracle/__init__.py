"""FP64 CPU oracle for the Lindblad-Magnus propagator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link
or execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do. It shares no code with the HIP path: it builds
its own operators from the scalar draws in ``synth`` and evaluates every step
in plain numpy float64 / complex128, in the order the paper states it:

* Eq. 8 Liouvillian, applied to the full H(t) of every evaluation point;
* Eq. 13 slice average (first-order Magnus) and the two-point Gauss-Legendre
  second-order Magnus term for piecewise-linear controls;
* Eq. 14 slice exponential by Taylor scaling and squaring (a deliberately
  different algorithm from the Pade approximant the GPU uses);
* Eq. 15 chain product, sequential left multiplication;
* process fidelity Re Tr(S_T^dagger U) / d^2 against S_T = conj(U_T) (x) U_T;
* exact adjoint gradient from the block-triangular Frechet derivative, central
  finite differences, and an RK4 integrator of Eq. 9;
* logical-subspace scores (Eq. 16-17) and the adjoint for any score of U;
* RK4 evolution of a state and the Uhlmann fidelity (the accuracy study);
* MLP and Adam references for the learned proposal and the optimiser;
* the closed-system reduction to Hilbert space (conj(V) (x) V) and the action
  of slice exponentials on a few columns, for superoperators too large for
  the dense path.
"""
from .model import (pauli, spin_op, exchange_terms, zeeman_terms, jump_ops,
                    hamiltonian)
from .liouville import vec, unvec, liouvillian, lift_hamiltonian
from .magnus import gl2_nodes, slice_omegas, slice_omega
from .expm import expm_taylor, frechet_block
from .optim import adam_project
from . import mlp
from . import logical
from . import states
from . import hilbert
from .propagator import (System, propagate, superop_of_unitary, fidelity,
                         grad_adjoint, grad_adjoint_at, grad_adjoint_seed, grad_adjoint_seed_at, grad_fd, grad_fd_cached, rk4_propagator,
                         slice_products)

__all__ = [n for n in dir() if not n.startswith("_")]
