"""MI355X-native periodic Stokes mobility solver (arXiv:1912.04501 hot path).

* ``spm``       - Python binding of the C ABI in ``include/spm.h`` (libspm.so, HIP for gfx950)
* ``workloads`` - seeded synthetic ellipse suspensions (inputs only)
* ``build``     - in-tree build of libspm.so
"""
