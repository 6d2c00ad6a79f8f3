"""CPU check that include/sem.h is a plain C99 interface: a C program that includes it compiles
with gcc in strict C99 mode, links against libsem.so and runs.  Without a GPU, sem_setup on a valid
descriptor must fail with a negative status and a message in sem_last_error(); with one (this test
is not marked gpu, so it normally runs where there is none) the program also runs the setup,
query and destroy cycle.  The program is started from a process that has not initialised the GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1806_01422_amd")
LIB = os.path.join(LIBDIR, "libsem.so")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "sem.h"

int main(void) {
  sem_ctx c = NULL;
  sem_desc d;
  int rc;
  const char* msg;
  int64_t ndof = 0, nodes = 0;
  memset(&d, 0, sizeof d);
  /* rejected before any device work: a null descriptor, then an order out of range */
  rc = sem_setup(NULL, NULL, &c);
  printf("null-desc %d %s\n", rc, sem_last_error());
  if (rc != SEM_ERR_ARG || c != NULL) return 2;
  d.dim = 3; d.elems[0] = 4; d.elems[1] = 1; d.elems[2] = 1; d.order = 99;
  d.length[0] = d.length[1] = d.length[2] = 1.0; d.nu = 0.01; d.dtype = SEM_F64; d.batch = 1;
  rc = sem_setup(&d, NULL, &c);
  printf("bad-order %d %s\n", rc, sem_last_error());
  if (rc >= 0) return 3;
  d.order = 7;
  rc = sem_setup(&d, NULL, &c);
  msg = sem_last_error();
  printf("setup %d %s\n", rc, msg);
  if (rc == SEM_OK) {
    if (sem_query(c, &ndof, &nodes) != SEM_OK || ndof != 3 * nodes || nodes != 28 * 7 * 7) return 4;
    if (sem_destroy(c) != SEM_OK) return 5;
    printf("device-cycle ok\n");
    return 0;
  }
  if (c != NULL || msg == NULL || strlen(msg) == 0) return 6;
  printf("no-device ok\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1806_01422_amd import build
        build.build()
    return LIB


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_plain_c99_caller(built, tmp_path):
    src = tmp_path / "caller.c"
    exe = tmp_path / "caller"
    src.write_text(PROGRAM)
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
           str(src), "-o", str(exe), "-L", LIBDIR, "-lsem", "-Wl,-rpath," + LIBDIR, "-Wl,--allow-shlib-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    lines = r.stdout.splitlines()
    assert lines[0].startswith("null-desc -1 ") and "descriptor" in lines[0]
    assert lines[1].startswith("bad-order -")
    assert lines[-1] in ("no-device ok", "device-cycle ok")
