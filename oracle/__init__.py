"""FP64 CPU oracle of iSIRA.  Test infrastructure only: imported by the tests, the smoke
check and the bench's CPU-baseline leg, never by the GPU library or its binding."""
