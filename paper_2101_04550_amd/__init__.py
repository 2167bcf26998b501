"""Extended lattice Boltzmann (LBGK) step on AMD MI355X: HIP kernels behind a C ABI.

The binding lives in ``paper_2101_04550_amd.elbm``; the library is built by
``paper_2101_04550_amd.build``. The request-serving loop lives in
``paper_2101_04550_amd.serving``.
"""
