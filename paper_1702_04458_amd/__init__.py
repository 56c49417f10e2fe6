"""MI355X-native decentralized baseband processing (arXiv:1702.04458).

Uplink detection by decentralized ADMM (Algorithm 1) and decentralized
conjugate gradients (Algorithm 2), downlink precoding by decentralized ADMM
(Algorithm 3), as hand-written HIP kernels for gfx950 behind the C ABI in
``include/dbp.h``.  ``paper_1702_04458_amd.api`` is a thin binding that takes
torch device tensors; importing this package loads nothing.
"""

__all__ = ["api", "inputs"]
