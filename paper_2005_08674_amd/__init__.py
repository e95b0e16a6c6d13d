"""MI355X-native D2Q9 lattice Boltzmann with the non-equilibrium symmetry boundary condition."""
