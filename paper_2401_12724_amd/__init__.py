"""BYSDF hot path for MI355X (gfx950)."""
