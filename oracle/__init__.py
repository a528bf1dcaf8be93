"""Plain FP64 CPU oracle for the PGCP hot path.  TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product: only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the GPU library (no kernels, headers, helpers or tables); the two
meet only at the seeded synthetic inputs in ``synth``.

Each module follows one step of Algorithm 3 (PGCP) of Choi, Leung-Liu, Gu and
Lui, "Parallelizable global conformal parameterization of simply-connected
surfaces via partial welding", written in the paper's order and notation:

  partition   Section 4.1 (cut edges -> face-graph components S_i)
  cotan       Section 4.2, cotangent Laplacian
  dncp        Section 4.2, DNCP local conformal parameterization
  weld        Section 3.4 (geodesic algorithm), Section 4.3.2 (Algorithms 1, 2),
              Section 4.4 (disk and sphere constraints)
  harmonic    Section 4.5, Laplace equation with the welded boundary
  sphere      Section 4.5, stereographic projection
  distortion  Section 5 angle distortion; Section 3.5 Beltrami coefficient
  pipeline    Algorithm 3 end to end

Sparse solves use scipy's SuperLU (dense numpy solve on tiny systems).
"""
