"""MI355X-native LSNIF query library (HIP kernels for gfx950 behind a C ABI).

``paper_2504_21627_amd.lsnif`` is the ctypes binding of ``include/lsnif.h``;
``paper_2504_21627_amd.serving`` builds per-request device buffers (windows of
a ray pool and their re-indexed pairs) for the serving loop; ``build`` compiles
the library with hipcc.
"""

from . import lsnif  # noqa: F401
