"""CPU oracle for the synthetic PIV image-pair generator -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
anything from here.  The product path (the HIP library and its Python binding)
never calls into this package, and this package never imports the product.

Two forms of the same computation live here:

* the float64 NumPy definition (``philox``, ``seed``, ``advect``, ``bins``,
  ``render``, ``epilogue``, ``grad``, ``pipeline``): plain, slow, written
  from the paper's model -- the single-particle Gaussian (Eq. 1), the particle
  sampling and masking rule and the flow mapping (Section 2, "Sampling the
  particles"), superposition (Section 2, "Considerations on the aggregation"),
  and the patch extent (Section 2, "Efficient rasterization");
* ``ra32``: a plain C mirror of the same steps in binary32 with every
  rounding spelled out, used wherever a float decides an integer (the 12-bit
  codes, the tile membership), so that both sides take that decision in the
  kernel's precision.

Each function states the passage of the paper it follows.  Readings of points
the paper leaves open are listed in the repository's design notes.
"""
