"""MI355X-native explicit filter and exact subgrid stress for wall-bounded channel flow.

The compute path lives in a HIP shared library (``csrc/``) behind a C ABI
declared in ``include/eles.h``; ``paper_1902_02508_amd.eles`` is its thin
ctypes binding. ``synth`` manufactures seeded synthetic inputs. Importing
the package itself loads nothing.
"""
