"""MI355X-native batched rigid-body step (Brax, arXiv 2106.13281) behind a C ABI."""
