"""MI355X-native Shan-Chen bubble growth / merging hot path (HIP kernels behind a C ABI)."""
