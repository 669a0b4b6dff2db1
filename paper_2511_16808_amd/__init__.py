"""MI355X (gfx950) Vanka-smoothed shifted-Laplacian multigrid Helmholtz solver.

The compute lives in libvh.so (HIP kernels + C++ runtime, C ABI in include/vh.h);
`binding` marshals torch GPU tensors to it.  Build with
`python -m paper_2511_16808_amd.build`.
"""
from . import binding  # noqa: F401
