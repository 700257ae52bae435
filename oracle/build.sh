#!/bin/sh
# Builds the CPU oracle (test infrastructure only) into oracle/liboracle.so.
set -e
cd "$(dirname "$0")"
gcc -O2 -std=gnu11 -fPIC -shared -ffp-contract=off -Wall -Wno-unused-function \
    -o liboracle.so core.c shower.c hard.c observables.c -lm -lpthread
