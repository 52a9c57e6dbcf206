"""MI355X-native Gerchberg-Saxton phase masks (method of alternating
projections) behind a C-ABI HIP library."""
