"""HEALPix Gaussian rasterizer for AMD Instinct MI355X (gfx950).

The forward and backward passes of the camera-agnostic 3D Gaussian
rasterizer on the HEALPix sphere grid (arXiv 2606.29794) run as hand-written
HIP kernels in ``libhp.so`` behind the C ABI of ``include/hp.h``.  This
package is the thin Python layer over it:

* ``_abi``    ctypes mirror of the C ABI (loading fails loudly if the
              library is missing -- there is no non-HIP path)
* ``raster``  buffer management with PyTorch tensors and the call sequence
* ``render``  ``torch.autograd.Function`` wrappers (render, HEALPix-SSIM loss)
* ``serve``   continuous-batching request loop
* ``scenes``  seeded synthetic workloads (inputs only)
* ``build``   hipcc build of libhp.so
"""

__all__ = ["_abi", "raster", "render", "serve", "scenes", "build"]
