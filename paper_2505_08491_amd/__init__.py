"""MI355X (gfx950) library for flexible GMRES on the coupled 3D-1D system with a
neural block preconditioner.

The compute path is the HIP library `libmdnp.so` (C ABI in include/mdnp.h);
this package holds its sources, build script and a thin Python binding.  The
binding is loaded on first use of one of its names, so that `build` can run
before the library exists.
"""
_API = ("Context", "HostSystem", "MdnpError", "N_WEIGHTS", "System", "host_assemble")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)


__all__ = list(_API)
