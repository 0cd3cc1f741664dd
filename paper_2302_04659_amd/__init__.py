"""MI355X-native MLS-MPM soft-body substep (HIP kernels behind a C ABI).

Importing the package is cheap: the HIP library is loaded on first use of
``paper_2302_04659_amd.mpm``.  ``paper_2302_04659_amd.scenes`` holds the
seeded synthetic inputs.
"""
