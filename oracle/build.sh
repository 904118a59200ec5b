#!/bin/bash
# Build the FP64 CPU oracle: plain C, IEEE-rounded in source order.
set -e
cd "$(dirname "$0")"
gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -fPIC -shared -Wall -Wextra \
    -o libgrmhd_oracle.so.tmp grmhd_oracle.c -lm
mv -f libgrmhd_oracle.so.tmp libgrmhd_oracle.so
