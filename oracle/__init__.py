"""CPU oracle of the ToF ReSTIR frame -- test infrastructure only."""
