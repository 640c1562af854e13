"""MI355X fine propagator for monolithic ALE fluid-structure interaction.

The numerical work runs in the HIP library libfsi.so (built in-tree by
``python -m paper_1907_01252_amd.build``); ``paper_1907_01252_amd.fsi`` is its
ctypes binding.  Importing the package loads nothing.
"""
