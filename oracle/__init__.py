"""FP64 CPU oracle of the OSCAR relaxation path -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never imports it."""
