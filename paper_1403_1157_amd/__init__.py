"""CDG2 operator for the six-species plaque model on MI355X (gfx950).

The compute path is the C-ABI library ``libcdg2.so`` built from ``csrc/``; the
Python binding in :mod:`paper_1403_1157_amd.cdg2` only marshals arguments.
"""
