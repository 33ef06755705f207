"""MI355X-native AMFR-W + sparse-grid combination solver for SABR-LMM PDEs (arXiv 2408.00559)."""
