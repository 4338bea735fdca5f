"""MI355X-native adjustable farthest point sampling (Li et al., arXiv 2208.08795).

Plain FPS (Algorithm 1), adjustable FPS with M storage sectors (Sec. III-B) and
nearest-point distance updating (Sec. III-C), as hand-written HIP kernels for
gfx950 behind the C ABI declared in ``include/afps.h``.  The Python functions
re-exported here only marshal torch tensors and streams into that ABI.
"""
__version__ = "0.1.0"

_BINDING_NAMES = ("fps", "afps", "afps_npdu", "batched", "BatchPlan", "library_path")


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
