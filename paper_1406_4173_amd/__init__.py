"""Exact betweenness with respect to a target set (Brandes++) on AMD MI355X.

The compute path is the HIP library ``libbcpp.so`` built from ``csrc/``; the Python
side in ``bcpp.py`` only marshals arguments to its C entry points. ``inputs`` draws
seeded synthetic graphs. Importing this package loads nothing; the library is loaded
on first use of ``paper_1406_4173_amd.bcpp``.
"""
