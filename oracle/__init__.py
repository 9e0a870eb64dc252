"""CPU reference ("oracle") for periodic frozen-density embedding.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 numpy
implementation of what the GPU library computes. Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never calls it and shares no code with it.

Modules follow Genova, Ceresoli & Pavanello, "Periodic Subsystem
Density-Functional Theory" (arXiv:1406.7803):

* ``dft``         naive separable discrete Fourier transforms (dense per-axis
                  DFT matrices), the transform pair of the plane-wave basis;
* ``basis``       cell, plane-wave spheres S_k, density sphere D;
* ``pseudo``      Gaussian local ions and Kleinman-Bylander projectors;
* ``hamiltonian`` H_I applied to bands (Eq. KS) and the explicit matrix;
* ``density``     subsystem densities (Sec. 2, BZ-integrated density);
* ``functionals`` Slater + Perdew-Zunger LDA, Thomas-Fermi x LC94 GGA KEDF
                  (Appendix, kinetic energy functional and potential);
* ``embed``       embedding potential in the recast form (Appendix, recast of
                  the effective potential) with Hartree from a Poisson solve;
* ``subspace``    residual, Teter-Payne-Allan preconditioner, Rayleigh-Ritz;
* ``occupations`` integer and Fermi-Dirac occupations (Sec. 2 and Sec. 3);
* ``scf``         the embedding cycle (Fig. 1b, one SCF step per cycle) and the
                  energies (Eq. for E_FDE, Appendix recast of the energy);
* ``mlp``         the FP64 reference of the learned preconditioner network.

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
