"""MI355X-native frequent-episode counting (non-overlapped occurrences of
serial episodes with inter-event delay intervals, two-pass elimination and
MapConcatenate segment counting), behind the C ABI declared in include/fe.h.

Submodules are imported on demand: ``paper_0905_2200_amd.fe`` binds the HIP
library, ``paper_0905_2200_amd.synth`` generates seeded synthetic inputs.
"""
__all__ = ["fe", "synth"]
