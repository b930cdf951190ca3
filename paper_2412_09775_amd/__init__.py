"""MI355X-native hot path of WaveOrder (arXiv 2412.09775).

The compute path is the HIP library ``libwaveorder.so`` (sources in
``csrc/``, C ABI in ``include/waveorder.h``); ``api`` is its thin ctypes
binding.  Build with ``paper_2412_09775_amd.build.build()``.
"""

from . import api  # noqa: F401
from .api import Optics  # noqa: F401
