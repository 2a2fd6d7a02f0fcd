"""Seeded synthetic inputs for the matrix power kernel.

This module only *builds inputs*: sparse matrices in CSR form and dense
vectors drawn from seeded generators.  It contains none of the arithmetic
of the method (no products, no level sets, no schedules), so both the
FP64 oracle and the HIP path may draw their inputs from it without
sharing any of the computation they are compared on.

The matrices stand in for the paper's benchmark set (Sec. 2, Table 2:
square sparse matrices of 0.6-1.6 M rows with 5-75 nonzeros per row and
more than 100 MB in CRS form), which is not available here:

* ``laplacian_2d`` / ``laplacian_3d``: Dirichlet 5- and 7-point stencils,
  natural (lexicographic) row order, integer entries.  The 3D one at 160^3
  has 6.96 nonzeros per row, the low end of Table 2.
* ``knn_graph_laplacian``: graph Laplacian of a symmetrised k-nearest-
  neighbour graph of uniform random points, shifted by ``shift * I``; an
  unstructured SPD matrix in the middle of Table 2's nonzeros-per-row range.
* ``random_pattern``: seeded random (possibly nonsymmetric, possibly
  disconnected) patterns for property tests.
* ``banded_random``: seeded random patterns inside a band, nonsymmetric
  unless asked otherwise, with long level structures.
"""
from .matrices import (  # noqa: F401
    CSR,
    laplacian_1d,
    laplacian_2d,
    laplacian_3d,
    knn_graph_laplacian,
    random_pattern,
    banded_random,
    block_diagonal,
    from_dense,
    identity,
    diagonal,
    cyclic_shift,
)
from .vectors import uniform_vector, integer_vector  # noqa: F401
