"""MI355X-native complex-to-complex 3D FFT (CROFT's method on one GPU)."""
