"""MI355X-native matched-filter trajectory search (arXiv:2209.09848).

The search itself runs in hand-written HIP kernels behind a C ABI
(include/tno_search.h, libtno_search.so); `tno` is its thin ctypes binding and
`synth` draws seeded synthetic inputs.
"""
