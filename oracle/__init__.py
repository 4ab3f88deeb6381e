"""CPU oracle of the monodomain FEM hot path (test infrastructure only)."""
