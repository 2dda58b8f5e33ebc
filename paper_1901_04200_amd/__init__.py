"""MI355X-native two-pass Monte Carlo adjoint calibration gradient."""
