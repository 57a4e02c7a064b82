"""Two-species multi-range Shan-Chen lattice Boltzmann on AMD MI355X (gfx950).

The compute path is the HIP library ``libsclbm.so`` built from ``csrc/``;
``sclbm`` is its thin ctypes binding.  Importing this package loads nothing;
``paper_0807_4471_amd.sclbm`` loads the library and fails loudly if it is
missing.
"""
