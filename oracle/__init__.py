"""CPU float64 oracle for the CTM environment of an iPEPS and its observables.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  The GPU library never calls
it, links it or falls back to it, and it shares no code with the GPU path.

Every function is written from the paper's statement of the method (sections,
equations and figure captions are cited in each docstring) in plain NumPy at
float64, with ``numpy.einsum`` / ``matmul`` / ``linalg.svd`` as the only
library steps.  Where the paper leaves a convention open, the reading taken is
stated next to the code that implements it.

Modules
-------
ctm     double-layer tensor, environment, enlarged corners, projectors,
        directional moves, sweeps, convergence and corner spectra
obs     norm per site, nearest-neighbour density matrices, energy, fidelity
models  ruby block-site Hamiltonian terms, Ising and product-state PEPS
mlp     reference multilayer perceptron for the learned warm start
"""
