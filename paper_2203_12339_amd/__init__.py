"""MI355X-native per-frame translucent transport (dipole + PCA + Haar PRT).

``tlt``       ctypes binding of libtlt.so (the C ABI in include/tlt.h).
``workloads`` builds a loaded renderer for a seeded synthetic workload.
``autograd``  torch.autograd.Function over render / render_backward.
"""
from . import tlt  # noqa: F401  (raises ImportError when libtlt.so is missing)
from .tlt import Renderer, prepare_scene  # noqa: F401
