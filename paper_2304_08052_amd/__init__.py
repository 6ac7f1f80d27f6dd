"""FRAM-RIR batched multi-channel RIR synthesis on MI355X (gfx950)."""
