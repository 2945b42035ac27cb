"""FP64 CPU oracle of the coupled colour-gradient LBM + DEM step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product library never imports it.
"""
