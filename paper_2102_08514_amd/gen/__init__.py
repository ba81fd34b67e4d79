"""Offline generator of the evaluation tables (exact rational analysis)."""
