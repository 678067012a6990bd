"""FP64 CPU oracle for certified one-sided Pompeiu-Hausdorff bounds.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg load it; the product path never does. It shares no code with
the HIP library. The arithmetic lives in hdo.c (plain C, double precision,
single-threaded); this module compiles it with gcc and marshals arguments.
`oracle.mlp` is the FP64 numpy oracle of the learned proposal's network and
features (forward, backward, Adam).
"""
from .hdo import (build, closest_point, point_soup, points_soup, Tree, bounds, bound, bound_u5, hausdorff,  # noqa: F401
                  HDO_OK, HDO_E_INVALID, HDO_E_CAPACITY, HDO_E_NOMEM, HDO_E_INTERNAL)
