"""MI355X-native grayscale morphological reconstruction and fill-holes.

The engine is the HIP library ``libmrecon.so`` (C ABI in include/mr.h);
``paper_1311_0378_amd.mrecon`` is its Python binding. Importing this package
loads nothing; the binding is imported on first attribute access, so the
seeded input generator (``paper_1311_0378_amd.synth``) can be used without it.
"""

_BINDING = ("recon_dilate", "fill_holes", "workspace_bytes", "read_counters", "make_tune",
            "default_tune", "MrError", "lib")


def __getattr__(name):
    if name in _BINDING:
        from . import mrecon
        return getattr(mrecon, name)
    raise AttributeError(name)
