"""MI355X-native two-component pseudopotential lattice Boltzmann step
(improved multicomponent Shan-Chen model of arXiv:2111.08666)."""
