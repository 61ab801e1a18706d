"""Surface hopping Gaussian beam ensemble on AMD Instinct MI355X (gfx950).

Hand-written HIP kernels behind the C ABI of ``include/shgb.h`` (libshgb.so);
``paper_1703_06116_amd.shgb`` is the Python binding (import it to load the
library; it raises if the library is not built), ``workloads`` the seeded
synthetic inputs, ``build`` the in-tree hipcc build.
"""
