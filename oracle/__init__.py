"""FP64 CPU oracle. Test infrastructure: only tests, the smoke check and the
benchmark's CPU-baseline leg may use it; the library never does."""
