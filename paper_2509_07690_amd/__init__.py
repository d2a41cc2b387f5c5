"""HYLU numerical factorisation and substitution on MI355X (gfx950)."""
