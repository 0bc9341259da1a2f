"""Plain FP64 CPU oracle for the Brillouin Dirac operator (Durr & Koutsou,
"Brillouin improvement for Wilson fermions", arXiv:1012.3615).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package:
only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import or call it.  It shares no code with the GPU library (no kernels,
headers, tables or helpers); the only common dependency is the ``synth``
module of seeded input generators, which holds none of the method's
arithmetic.

Every function is written from the paper's definitions, in numpy, in FP64,
without blocking or fusion:

* ``constants``   - stencil weights of the Brillouin Laplacian and the
  isotropic derivative derived from their momentum-space product forms
  (Sec. 4.1, Eqs. def_4Dbri and the isotropic derivative of App. C), and the
  resulting (rho_k, lambda_k) of Tab. rholambda;
* ``gamma``       - a Hermitian chiral basis of the Euclidean gamma matrices;
* ``transporters``- W(x, x+n) as the average over all shortest lattice paths
  (Sec. 5.1), by explicit path enumeration;
* ``dirac``       - D = sum_mu gamma_mu nabla^iso_mu - (1/2) Lap^bri + m
  (Eq. def_pref with c_SW = 0), its adjoint, a pointwise (sampled-site)
  version and the dense matrix for small lattices;
* ``factorized``  - an independent second formulation of the same operator as
  ordering-averaged products of one-dimensional covariant hop operators
  (the factorisation of App. D applied to the product forms), used as a pin;
* ``free``        - the free-field momentum-space symbol and propagator;
* ``solver``      - CG on the normal equations;
* ``grad``        - gradients of Re<chi, D psi> with respect to links and psi;
* ``projection``  - the projections to U(3) and SU(3) of Sec. 5.2 (SVD, then
  the constrained phase maximisation);
* ``smearing``    - one APE smearing step (Eq. def_ape);
* ``clover``      - the clover term of Eq. def_pref (clover-leaf field strength);
* ``production``  - the operator of Sec. 5: back-projected transporters plus
  the clover term;
* ``overlap``     - the overlap operator with the Brillouin kernel (Sec. 7),
  dense and exact for tiny lattices;
* ``ultralocal``  - the generic class of Sec. 8 with any (lambda_k, rho_k)
  table (Tab. rholambda: Wilson, hypercube, Brillouin columns).

Parity status of each function is listed in the module docstrings.
"""
from . import (constants, gamma, lattice, transporters, dirac, factorized, free, solver, grad,  # noqa: F401
               projection, smearing, clover, production, overlap, ultralocal)
