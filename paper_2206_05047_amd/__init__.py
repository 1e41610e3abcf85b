"""MI355X-native ADMM light-field super-resolution (arXiv 2206.05047)."""
