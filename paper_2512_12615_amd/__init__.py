"""Device-side eBPF runtime for MI355X (gfx950)."""
