"""MI355X-native LSNIF query library (HIP kernels for gfx950 behind a C ABI).

``paper_2504_21627_amd.lsnif`` is the ctypes binding of ``include/lsnif.h``;
``paper_2504_21627_amd.runtime`` adds a small convenience layer over it.
"""

from . import lsnif  # noqa: F401
