"""MI355X-native batched Annealed Stein ICP (arXiv 2412.08346)."""
