#!/bin/sh
# Builds the CPU oracle (test infrastructure only) as liboracle.so.
# Plain FP64, no SIMD intrinsics, no FMA contraction.
set -e
cd "$(dirname "$0")"
g++ -std=c++17 -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared -Wall -Wno-unused-function \
    -o liboracle.so orc_kinetic.cpp orc_mesh.cpp orc_solver.cpp
