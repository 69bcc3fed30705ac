"""FP64 CPU oracle for the SAR Range Doppler Algorithm and its image-quality
metrics.  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and
the benchmark's CPU-baseline leg, never by the product path."""
