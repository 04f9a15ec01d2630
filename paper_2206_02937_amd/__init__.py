"""MI355X-native Compton-scattering Monte-Carlo step with a learned sampler.

The compute lives in ``libcompton.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/compton.h``); ``paper_2206_02937_amd.compton`` is the
ctypes binding.  Nothing is imported here, so that the input generators in
``paper_2206_02937_amd.plasma`` can be used without loading the GPU library.
"""
