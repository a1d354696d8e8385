"""MI355X-native single-chain-in-mean-field Monte-Carlo sweep (HIP for gfx950)."""
