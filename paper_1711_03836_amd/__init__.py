"""MI355X-native even-odd Wilson-clover operator and CG (BQCD hot path)."""
