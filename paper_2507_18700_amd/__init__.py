"""MI355X-native VMC hot path for GRU RNN wave functions."""
