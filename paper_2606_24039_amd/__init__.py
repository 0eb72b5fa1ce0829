"""MI355X-native batched SQP-ADMM solver for optimal-control QPs.

The solve runs in the HIP library `libocp_admm.so` (built in-tree by
`paper_2606_24039_amd.build`); this package only marshals arguments.
"""
from ._abi import default_settings, lib  # noqa: F401

__all__ = ["default_settings", "lib"]
