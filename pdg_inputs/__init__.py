"""Seeded synthetic inputs shared, as data only, by the oracle and the HIP path.

This package generates meshes, partitions, tissue tensors, parameter tables
and piecewise-constant initial data.  It holds none of the method's arithmetic
(no basis, quadrature, assembly, ionic model, preconditioner or solver).
"""
from .meshdata import Mesh  # noqa: F401
from . import params  # noqa: F401
