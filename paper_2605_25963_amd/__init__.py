"""MI355X (gfx950) photon transport through closed triangle meshes for HPGe
full-energy-peak efficiency calibration, after DetMesh-Gadep (arXiv 2605.25963).

The work runs in hand-written HIP kernels in libgadep.so behind the C
interface include/gadep.h; gadep.py is its ctypes binding and autograd.py
the torch.autograd wrapper of the score-function gradient.
"""
from . import gadep  # noqa: F401
from .gadep import Context, GadepError, load_workload, mesh_prepare  # noqa: F401
