"""Sorting-based median filter (arXiv:1406.1717) on AMD MI355X (gfx950)."""
