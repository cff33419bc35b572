"""Named workloads (placeholder, filled in below)."""
