"""MI355X (gfx950) HSDE-ADMM solver for SOS-derived SDPs.

The solver lives in the HIP library libsos.so (C ABI: include/sos.h); the
`binding` module marshals Python arguments into it.  Import `binding` to use it:
it raises if the library has not been built.
"""
__all__ = ["binding"]
