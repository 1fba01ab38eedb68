"""MI355X (gfx950) implementation of the fused stream-and-collide sweep of the
binary free-energy lattice Boltzmann method of Pooley, Kusumaatmaja and Yeomans
(arXiv:0812.1282): HIP kernels behind the C ABI of include/lb.h, with a thin
ctypes binding in `lbm` and seeded synthetic inputs in `workloads`."""
