"""FBPQ query-time search on AMD MI355X (gfx950): HIP kernels behind a C ABI.

The compute lives in libfbpq.so (built from csrc/ by paper_1404_1831_amd.build);
`fbpq` is its ctypes binding.
"""
