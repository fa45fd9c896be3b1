"""MI355X-native hot path of the time-resolved channel DNS (arxiv 1808.06461).

The compute lives in the HIP library ``libchn.so`` (sources in ``csrc/``, C ABI
in ``include/chn.h``); ``chn`` is its ctypes binding.
"""
from .chn import Channel, ChnError, header_symbols, lib  # noqa: F401
