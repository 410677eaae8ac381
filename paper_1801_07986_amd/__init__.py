"""MI355X-native limited-1PN direct N-body hot path (placeholder; binding added below)."""
