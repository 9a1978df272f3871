"""FP64 brute-force oracle of the Pulsar sphere renderer (test infrastructure only)."""
