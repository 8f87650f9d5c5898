"""MI355X-native coupled ternary phase-field LB step (arXiv 2311.05091)."""
