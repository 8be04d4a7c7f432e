"""MI355X-native exact t-SNE hot path (affinities + exact gradient iteration).

The compute path is libtsne355.so (hand-written HIP kernels for gfx950)
behind the C ABI of ``include/tsne355.h``; ``_lib`` binds it with ctypes and
``tsne.ExactTSNE`` drives it. ``synth`` holds the seeded input generators.
Submodules are imported lazily so that importing the package does not load
the GPU library.
"""
__all__ = ["synth", "tsne", "_lib", "build"]
