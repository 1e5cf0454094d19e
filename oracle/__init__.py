"""CPU oracle (test infrastructure only): plain FP64 reference of the LETKF
analysis and of the brute-force Kalman filter that pins it.  Only tests/, the
smoke check and the bench's CPU-baseline leg use it; the GPU library never does."""
