"""Plain, slow, CPU reference ("oracle") for the randomized Gram-Schmidt path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call or link anything in this package.  Only the
test-suite, the smoke check in __graft_entry__.py and the CPU-baseline leg
of the benchmark use it.

It follows Balabanov & Grigori, "Randomized Gram-Schmidt process with
application to GMRES" (arXiv:2011.05090):

* ``philox``  -- the counter-based generator behind every random sketch
  (Salmon et al., SC'11), from its published definition.
* ``sketch``  -- the sketching operators of Sec. 2.1: Gaussian, (P-)SRHT,
  identity; dense materialisation for small sizes.
* ``rgs``     -- Algorithm 2 (RGS) and the classical projectors of Sec. 1.2
  (CGS, CGS2, MGS) used as pins and stability references.
* ``stencil`` -- the 7-point convection-diffusion operator used as the Arnoldi
  mat-vec.
* ``gmres``   -- Algorithm 3 (RGS-Arnoldi) and randomized GMRES (Sec. 4.2).
* ``metrics`` -- the quantities the paper reports (Delta_m, tilde Delta_m,
  cond, omega and its certified bound of Prop. 3.7).

Arithmetic is fp64 unless a function's ``precision`` argument asks for the
paper's multi-precision model (Sec. 2.3, the paragraph after Algorithm 2), in
which case the high-dimensional projection (step 3) and the storage of W and
Q are emulated in float32 while everything else stays in fp64.
"""

from . import philox, sketch, rgs, stencil, gmres, metrics  # noqa: F401
