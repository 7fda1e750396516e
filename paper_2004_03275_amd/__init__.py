"""MI355X-native block-forest finite-volume update (MPI-AMRVAC hot path)."""
