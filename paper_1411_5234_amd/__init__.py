"""MI355X-native direct N-body hot path (Hermite-4, block time steps, HIP kernels).

Submodules: `inputs` (seeded initial conditions), `_lib` (ctypes binding of
libnbody.so), `nbody` (device state, context, block-step driver), `serve`
(continuous-batching ensemble server), `build` (hipcc build of the library).
Nothing is imported eagerly, so `inputs` can be used without torch or a GPU.
"""
__version__ = "0.1.0"
