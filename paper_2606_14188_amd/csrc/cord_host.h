// Host-side helpers shared by the simulator API and the planning server.
#pragma once
#include "../../include/cord.h"
#include "cord_internal.h"

namespace cord {
int validate(const cord_instance_desc& d, int i);
void fill_instdev(const cord_instance_desc& d, InstDev& I);
int bucket_of(int topo, int n);
int default_config(int topo, int nmax);
int set_error(int code, const char* msg);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
struct KArgs;
// Optional device scratch for a linearize launch: get(ctx, floats) returns a
// buffer of at least that many floats that no other work uses until the
// launch ends, or null (the kernel then works without it).
struct KeptSource {
    float* (*get)(void* ctx, size_t floats);
    void* ctx;
};
// penalty / fric: some instance of the launch uses the penalty grasp / has
// friction (mu > 0); either rules out the banded direct kernel, and fric
// selects the kernels compiled with the friction cone.
hipError_t launch_linearize(int cfg_index, int topo, int nmax, bool penalty, bool fric, const KArgs& a, int nblk,
                            int tmax, hipStream_t st, const KeptSource& ks);
}  // namespace cord
