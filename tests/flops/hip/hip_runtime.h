// empty stand-in: the physics header is compiled on the host for counting
