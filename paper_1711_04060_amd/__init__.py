"""MI355X-native Poisson-Fermi hot path (arXiv:1711.04060)."""
