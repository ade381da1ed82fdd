"""MI355X-native pressure-correction step of a one-fluid two-phase solver."""
