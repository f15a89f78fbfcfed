"""MI355X-native 3D Voronoi / power diagram construction."""
