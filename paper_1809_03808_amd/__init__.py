"""MI355X-native FFT-based fast direct solver for the separable FE Helmholtz
problem with first-order absorbing boundary conditions (Toivanen & Wolfmayr).

The solver lives in the HIP library ``libhelm.so`` (C ABI, ``include/helm.h``);
``paper_1809_03808_amd.helm`` is its thin ctypes binding.  Importing this
package does not load the library; ``paper_1809_03808_amd.helm.lib()`` does and
raises if it has not been built.
"""

__all__ = ["helm", "inputs"]
