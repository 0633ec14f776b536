"""Poisson-disk point-cloud decimation on one MI355X (gfx950, HIP).

The GPU path lives in the C-ABI library ``libpdd.so`` (built from ``csrc/``);
``paper_2311_17604_amd.pdd`` is its thin ctypes binding.  Importing this
package does not load the library; ``scangen`` is the seeded input generator.
"""
