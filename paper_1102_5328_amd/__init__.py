"""MI355X-native tile Householder QR with an empirical (NB, IB) autotuner."""
