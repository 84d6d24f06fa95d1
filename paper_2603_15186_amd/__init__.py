"""MI355X-native forward renderer for hierarchical 3D Gaussian Splatting scenes."""
