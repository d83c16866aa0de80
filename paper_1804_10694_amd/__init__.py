"""tgemm: generalized matrix multiply C = alpha*A*B + beta*C on AMD MI355X (gfx950).

The computation is the one the Tiramisu paper (Section I) uses as its running
example of a kernel worth a compiler's effort; the library applies the
transformations the paper lists for it (two-level tiling, array packing,
register blocking, full/partial tile separation, autotuned tile sizes) in
hand-written HIP for gfx950, behind the C ABI declared in include/tgemm.h.

Importing the package loads nothing.  `paper_1804_10694_amd.tgemm` loads the
HIP library and raises if it is not built; there is no CPU fallback.
`paper_1804_10694_amd.inputs` holds the seeded input generators only.
"""
__all__ = ["tgemm", "inputs"]
