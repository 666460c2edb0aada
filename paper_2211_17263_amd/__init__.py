"""MI355X-native plateau-reduced gradient estimator."""
