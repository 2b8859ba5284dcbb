"""MI355X-native coupled reactive-transport lattice Boltzmann step (lbrx)."""
