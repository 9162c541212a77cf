"""stockfft for MI355X: batched complex-to-complex FP32 FFTs on gfx950."""
