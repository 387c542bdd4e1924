"""The C ABI from C: a C99 program that includes include/dloc.h and links
libdloc.so compiles warning-free under -pedantic, and its host-only calls
(version, defaults, weights inspection, argument rejection) behave as the
header states.  No GPU is touched."""
import os
import subprocess

import pytest

import smlm_synth as S

dl = pytest.importorskip("paper_2410_02314_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROGRAM = r"""
#include <stdio.h>
#include <stdlib.h>
#include "dloc.h"

int main(int argc, char **argv)
{
    if (argc != 2) return 90;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 91;
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    unsigned char *blob = malloc((size_t)n);
    if (!blob || fread(blob, 1, (size_t)n, f) != (size_t)n) return 92;
    fclose(f);

    dl_config cfg;
    if (dl_default_config(&cfg) != DL_OK) return 1;
    dl_net_info info;
    if (dl_inspect_weights(blob, (size_t)n, &info) != DL_OK) return 2;
    double rate = 0.0;
    int bad_rate = dl_measure_rate(99, 0, 1, &rate);
    int bad_info = dl_inspect_weights(blob, (size_t)n - 4, &info);
    int null_net = dl_set_camera_maps(NULL, NULL, NULL, 0, 0);
    dl_net_info ok;
    dl_inspect_weights(blob, (size_t)n, &ok);
    printf("abi=%u precision=%d threshold=%.2f C=%d nblocks=%d head=%d radius=%d "
           "bad_rate=%d bad_info=%d null_net=%d\n",
           dl_abi_version(), cfg.precision, cfg.threshold, ok.C, ok.nblocks, ok.head_outputs,
           ok.receptive_radius, bad_rate, bad_info, null_net);
    free(blob);
    return 0;
}
"""


def test_c_program_uses_the_abi(tmp_path):
    src = tmp_path / "abi.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.dirname(dl.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(exe), "-L", libdir, "-ldloc", f"-Wl,-rpath,{libdir}",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    spec, w = S.make_net("BU", 2)
    blob = tmp_path / "bu.dlw"
    blob.write_bytes(S.serialize_weights(spec, w))
    out = subprocess.run([str(exe), str(blob)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    fields = dict(kv.split("=") for kv in out.stdout.split())
    assert fields["abi"] == "3" and fields["precision"] == "0" and fields["threshold"] == "0.30"
    assert (fields["C"], fields["nblocks"], fields["head"], fields["radius"]) == ("48", "5", "10", "63")
    assert int(fields["bad_rate"]) == dl.DL_ERR_INVALID_ARG
    assert int(fields["bad_info"]) == dl.DL_ERR_BAD_WEIGHTS
    assert int(fields["null_net"]) == dl.DL_ERR_INVALID_ARG
