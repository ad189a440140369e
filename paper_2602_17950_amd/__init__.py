"""MI355X-native ground-state solver for rotating spin-orbit-coupled spin-1
condensates (Fourier-spectral PCG of arXiv 2602.17950).

``paper_2602_17950_amd.gs`` is the Python binding of the C-ABI library
``libgs.so`` (hand-written HIP kernels for gfx950); ``inputs`` builds seeded
synthetic problems and initial guesses. Importing the package does not load the
library; ``gs`` loads it on first use and raises if it is missing.
"""
