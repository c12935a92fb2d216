"""MI355X-native entropic unbalanced optimal transport (generalized Sinkhorn scaling)."""
