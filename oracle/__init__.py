"""TEST INFRASTRUCTURE ONLY.

FP64 CPU oracle for the doubly-periodic spectral Ewald (DP-SE) solve of
Maxian, Pelaez, Greengard and Donev, "A fast spectral method for electrostatics
in doubly-periodic slit channels" (arXiv 2101.07088), plus an independent
Ewald2D + image-series reference.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything here. The product path (the HIP library and
its Python binding) never imports, calls or links this package, and this
package never imports the product.
"""
