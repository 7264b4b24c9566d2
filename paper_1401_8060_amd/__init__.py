"""MI355X-native track search of all-sky seedless clustering (arXiv:1401.8060).

The compute lives in libstt.so (HIP, gfx950) behind the C ABI of include/stt.h;
``paper_1401_8060_amd.stt`` is its Python binding.
"""
