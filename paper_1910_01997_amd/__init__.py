"""MI355X (gfx950) surfel Gauss-Newton library: C ABI over hand-written HIP
kernels (libsurfgn.so), a ctypes binding (surfgn), the keyframe-batch engine
and the serving loop.  Importing the package loads nothing; the binding loads
the compiled library on first use and fails loudly if it is missing."""

__all__ = ["surfgn", "engine", "serve"]
