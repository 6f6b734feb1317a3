"""Plain FP64 CPU oracle for FIRM (Wang, Shkolnisky & Singer, "A Fourier-based
Approach for Iterative 3D Reconstruction from Cryo-EM Images").

TEST INFRASTRUCTURE ONLY.  Nothing in the library package imports, links or
runs anything under this directory; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark do.  The oracle shares no code, tables,
constants or helpers with the HIP path.

Every function writes out the definition it follows (the paper's equations,
cited by section and equation label) in the most direct form numpy allows:
separable phase tables and library matrix products are the only shortcuts, and
none of them reorders or approximates the sums.  There is no non-uniform FFT
here: every sum the GPU evaluates with gridding is evaluated directly.

Modules
  firm     geometry, forward projector A, back-projector A*, convolution
           kernel Ker, Toeplitz / circulant-embedded products, CG and PCG,
           dense solve, Krylov-subspace reference iterate, FSC.
  blobs    closed-form Gaussian-blob volumes, their Fourier slices and their
           real-space projections (projection-slice theorem, section 3.1).
  pcnet    the preconditioner conv net in FP64 with hand-written gradients.
  direct   ctypes binding of direct.c: the same direct sums in plain C for
           sampled outputs at large sizes.

Readings of the paper where it is silent or garbled are listed in the module
docstrings where they are used.
"""
