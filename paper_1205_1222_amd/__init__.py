"""MI355X (gfx950) regular force of the Ahmad-Cohen neighbour scheme.

The GPU library is ``libnb6.so`` (C ABI in ``include/nb6.h``); ``nb6`` is its
ctypes binding.  Build with ``python -m paper_1205_1222_amd.build``.
"""
