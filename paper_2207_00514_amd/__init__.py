"""MI355X-native single-tree Boruvka EMST (placeholder, filled in below)."""
