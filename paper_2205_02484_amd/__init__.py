"""MI355X-native HARM-style GR-MHD time step (after the cuHARM paper, arXiv 2205.02484).

The compute path is the HIP library libgrmhd.so behind the C ABI in include/grmhd.h; the
Python modules here marshal arguments (`grmhd`), build synthetic inputs (`torus_init`,
`workloads`) and run the ensemble request loop (`serve`).  Importing the package does not
load the library; `paper_2205_02484_amd.grmhd` does, and fails loudly when it is missing.
"""
