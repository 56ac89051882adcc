"""FP64 CPU oracle of the matched-filter trajectory search -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the HIP library and never imports it.
"""
