"""Singular value soft-thresholding through the polar decomposition, on MI355X."""
