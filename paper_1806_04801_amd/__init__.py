"""MI355X-native hot path of the harmonic surface mapping algorithm (HSMA)."""
