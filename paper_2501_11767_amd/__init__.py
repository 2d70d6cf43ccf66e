"""MI355X (gfx950) solver for the linear systems of the semi-implicit
Cahn-Hilliard / Allen-Cahn / Navier-Stokes time step of arXiv 2501.11767.

``chns``    ctypes binding of the C-ABI library libchns.so (include/chns.h).
``inputs``  seeded synthetic initial data and workload parameters.
``build``   in-place hipcc build of the library.

Submodules are imported on demand so that ``inputs`` can be used without
loading the GPU library.
"""
