"""MI355X (gfx950) vacancy-jump AKMC: HIP library libakmc.so behind the C
interface of include/akmc.h, its Python binding (akmc) and seeded
synthetic workloads (workloads)."""
