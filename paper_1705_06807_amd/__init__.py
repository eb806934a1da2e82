"""ParRep (parallel replica dynamics) for bistable CTMC reaction networks on MI355X.

The compute path is a HIP library (``libparrep.so``) behind a C ABI declared in
``include/parrep.h`` and ``include/parrep_estimate.h``;
:mod:`paper_1705_06807_amd.binding` marshals arguments to it.
Importing this package does not load the library; the first call does, and fails
loudly if it has not been built.
"""

__all__ = ["workloads", "binding"]
