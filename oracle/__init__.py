"""FP64 CPU oracle for the channel RK3 hot path and the low-storage filter stage.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU-baseline leg may import or run anything in this package.
The GPU path (``paper_1808_06461_amd``) never imports it, and this package
never imports the GPU path; the two share only the seeded input generators in
``synth``.

Every routine here is a plain, slow restatement of the method as the paper
describes it (Appendix A: velocity-vorticity formulation and semi-implicit
RK3; Appendix B: compact finite differences and the homogeneous Helmholtz
problem; Section 3.1: sharp Fourier cut-off filter, filtered stresses and the
SGS tensor), in float64, with numpy/scipy library primitives (FFTs, dense
solves) as steps.  The pins that tie each part to the paper or to closed-form
mathematics live in ``tests/test_oracle_*.py``.
"""
