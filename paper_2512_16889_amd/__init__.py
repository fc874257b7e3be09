"""MI355X (gfx950) scattered-wave-function solver for strong-field pair production.

The hot path (RK4 stepping of the scattered Dirac wave with pseudo-spectral
derivatives, the source term, the boundary mask and the amplitude reductions)
runs in the HIP library ``libswf.so`` behind the C ABI of ``include/swf.h``;
``paper_2512_16889_amd.swf`` is its ctypes binding.
"""
__all__ = ["swf", "build"]
