"""MI355X-native exact pan-matrix-profile motif search (HIP/gfx950)."""
