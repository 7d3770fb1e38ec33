"""rhipm: condensed reduced-space interior-point KKT hot path on AMD MI355X.

The compute path is the HIP library librhipm.so (include/rhipm.h); this
package only builds it and marshals arguments to it.
"""
from .api import Net, Symbolic, lib  # noqa: F401
